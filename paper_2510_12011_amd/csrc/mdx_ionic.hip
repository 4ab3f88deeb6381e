// Pointwise ionic-model kernels: one thread per mesh node, states stored
// structure-of-arrays (u[s * ld + i]) so every state load/store of a
// wavefront is one contiguous segment.
//
// The operator split of the paper's Eq. (2): states advance from (V^k, u^k)
// (gating variables by Rush-Larsen y <- y_inf + (y - y_inf) exp(-dt/tau),
// the other states by forward Euler), then the current is evaluated at
// (V^k, u^{k+1}).  Currents are per unit capacitance (pA/pF = mV/ms); the
// tissue's Cm (uF/mm^2) turns them into uA/mm^2.
//
// Models (the paper names them without equations; written from the original
// publications):
//  * Mitchell-Schaeffer two-variable model (Bull. Math. Biol. 2003), with the
//    membrane variable u = (V - v_rest) / v_amp and gate h;
//  * ten Tusscher-Panfilov 2006 human ventricular model, endocardial cell
//    (Am. J. Physiol. Heart Circ. Physiol. 291:H1088), 18 states + V.
#include "mdx_internal.h"

namespace mdx {

namespace {

enum { MDX_KIND_NONE = 0, MDX_KIND_MS = 1, MDX_KIND_TT = 2 };
constexpr int MS_NP = 7;
constexpr int TT_NS = 18;
constexpr int TT_NP = 12;

struct IonicParams {
    double v[16];
};

// ---------------------------------------------------------------------------
// Mitchell-Schaeffer: params tau_in, tau_out, tau_open, tau_close, u_gate,
// v_rest, v_amp.  dh/dt = (1-h)/tau_open below u_gate, -h/tau_close above;
// I_ion/Cm = -v_amp (h u^2 (1-u)/tau_in - u/tau_out).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double ms_point(const IonicParams &P, double dt, double V, double &h)
{
    const double tau_in = P.v[0], tau_out = P.v[1], tau_open = P.v[2], tau_close = P.v[3];
    const double u_gate = P.v[4], v_rest = P.v[5], v_amp = P.v[6];
    double u = (V - v_rest) / v_amp;
    bool recovering = u < u_gate;
    double h_inf = recovering ? 1.0 : 0.0;
    double tau = recovering ? tau_open : tau_close;
    h = h_inf + (h - h_inf) * exp(-dt / tau);
    return -v_amp * (h * u * u * (1.0 - u) / tau_in - u / tau_out);
}

// ---------------------------------------------------------------------------
// ten Tusscher-Panfilov 2006, endocardial.
// State slots: Ki Nai Cai CaSR CaSS Rbar | xr1 xr2 xs m h j d f f2 fCass s r
// Params: GNa GK1 Gto GKr GKs GCaL GbNa GbCa GpCa GpK PNaK kNaCa
// ---------------------------------------------------------------------------
enum { KI, NAI, CAI, CASR, CASS, RBAR, XR1, XR2, XS, MG, HG, JG, DG, FG, F2G, FCASS, SG, RG };

// cell and environment constants
constexpr double Rgas = 8314.472, Temp = 310.0, Far = 96485.3415;
constexpr double RTONF = Rgas * Temp / Far;
constexpr double CAPAC = 0.185, VOLC = 0.016404, VOLSR = 0.001094, VOLSS = 0.00005468;
constexpr double K_O = 5.4, NA_O = 140.0, CA_O = 2.0;
constexpr double P_KNA = 0.03, KM_K = 1.0, KM_NA = 40.0, KM_NAI = 87.5, KM_CA = 1.38;
constexpr double K_SAT = 0.1, NCX_GAMMA = 0.35, NCX_ALPHA = 2.5, K_PCA = 0.0005;
constexpr double BUF_C = 0.2, KBUF_C = 0.001, BUF_SR = 10.0, KBUF_SR = 0.3;
constexpr double BUF_SS = 0.4, KBUF_SS = 0.00025;
constexpr double VMAX_UP = 0.006375, K_UP = 0.00025, V_REL = 0.102;
constexpr double K1_PRIME = 0.15, K2_PRIME = 0.045, K3 = 0.06, K4 = 0.005;
constexpr double EC_SR = 1.5, MAX_SR = 2.5, MIN_SR = 1.0;
constexpr double V_LEAK = 0.00036, V_XFER = 0.0038;

constexpr double TT_V_REST = -85.23;
__constant__ double TT_U0[TT_NS] = {136.89,   8.604,    0.000126, 3.64,   0.00036, 0.9073,
                                    0.00621,  0.4712,   0.0095,   0.00172, 0.7444, 0.7045,
                                    3.373e-5, 0.7888,   0.9755,   0.9953, 0.999998, 2.42e-8};

// factors of the currents that depend on V only
struct VOnly {
    double ical_drive;   // 2F * w/expm1(w) with w = 2(V-15)F/RT
    double ical_ew;      // exp(w)
    double nak_den;      // 1 + 0.1245 e^{-0.1 VF/RT} + 0.0353 e^{-VF/RT}
    double ncx_up, ncx_down, ncx_sat;   // e^{g VF/RT}, e^{(g-1) VF/RT}, 1 + ksat e^{(g-1)VF/RT}
    double ipk;          // 1 / (1 + exp((25 - V)/5.98))
};

__device__ __forceinline__ VOnly v_only(double V)
{
    VOnly o;
    double w = 2.0 * (V - 15.0) / RTONF;
    o.ical_ew = exp(w);
    o.ical_drive = 2.0 * Far * (w == 0.0 ? 1.0 : w / expm1(w));
    double phi = V / RTONF;
    o.nak_den = 1.0 + 0.1245 * exp(-0.1 * phi) + 0.0353 * exp(-phi);
    o.ncx_up = exp(NCX_GAMMA * phi);
    o.ncx_down = exp((NCX_GAMMA - 1.0) * phi);
    o.ncx_sat = 1.0 + K_SAT * o.ncx_down;
    o.ipk = 1.0 / (1.0 + exp((25.0 - V) / 5.98));
    return o;
}

struct Currents {
    double iK1, ito, iKr, iKs, iCaL, iNaK, iNa, ibNa, iNaCa, ibCa, ipK, ipCa;
    __device__ double total() const
    {
        return iK1 + ito + iKr + iKs + iCaL + iNaK + iNa + ibNa + iNaCa + ibCa + ipK + ipCa;
    }
};

__device__ __forceinline__ Currents tt_currents(const IonicParams &P, double V, const VOnly &vo,
                                                const double *y)
{
    const double gNa = P.v[0], gK1 = P.v[1], gto = P.v[2], gKr = P.v[3], gKs = P.v[4];
    const double gCaL = P.v[5], gbNa = P.v[6], gbCa = P.v[7], gpCa = P.v[8], gpK = P.v[9];
    const double pNaK = P.v[10], kNaCa = P.v[11];
    const double ki = y[KI], nai = y[NAI], cai = y[CAI];
    const double e_k = RTONF * log(K_O / ki);
    const double e_na = RTONF * log(NA_O / nai);
    const double e_ks = RTONF * log((K_O + P_KNA * NA_O) / (ki + P_KNA * nai));
    const double e_ca = 0.5 * RTONF * log(CA_O / cai);
    const double ko_scale = sqrt(K_O / 5.4);
    Currents c;
    // inward rectifier: steady-state rectification a/(a+b)
    double a_k1 = 0.1 / (1.0 + exp(0.06 * (V - e_k - 200.0)));
    double b_k1 = (3.0 * exp(0.0002 * (V - e_k + 100.0)) + exp(0.1 * (V - e_k - 10.0)))
                / (1.0 + exp(-0.5 * (V - e_k)));
    c.iK1 = gK1 * ko_scale * (a_k1 / (a_k1 + b_k1)) * (V - e_k);
    c.ito = gto * y[RG] * y[SG] * (V - e_k);
    c.iKr = gKr * ko_scale * y[XR1] * y[XR2] * (V - e_k);
    c.iKs = gKs * y[XS] * y[XS] * (V - e_ks);
    double m = y[MG];
    c.iNa = gNa * m * m * m * y[HG] * y[JG] * (V - e_na);
    c.ibNa = gbNa * (V - e_na);
    c.iCaL = gCaL * y[DG] * y[FG] * y[F2G] * y[FCASS] * vo.ical_drive
           * (0.25 * y[CASS] * vo.ical_ew - CA_O);
    c.ibCa = gbCa * (V - e_ca);
    c.iNaK = pNaK * (K_O / (K_O + KM_K)) * (nai / (nai + KM_NA)) / vo.nak_den;
    constexpr double nao3 = NA_O * NA_O * NA_O;
    constexpr double ncx_den = (KM_NAI * KM_NAI * KM_NAI + nao3) * (KM_CA + CA_O);
    c.iNaCa = kNaCa * (vo.ncx_up * nai * nai * nai * CA_O - vo.ncx_down * nao3 * cai * NCX_ALPHA)
            / (ncx_den * vo.ncx_sat);
    c.ipCa = gpCa * cai / (K_PCA + cai);
    c.ipK = gpK * vo.ipk * (V - e_k);
    return c;
}

__device__ __forceinline__ double rush_larsen(double y, double y_inf, double tau, double dt)
{
    return y_inf - (y_inf - y) * exp(-dt / tau);
}

__device__ __forceinline__ double sq(double x) { return x * x; }

__device__ double tt_point(const IonicParams &P, double dt, double V, double *y)
{
    const VOnly vo = v_only(V);
    const Currents c = tt_currents(P, V, vo, y);

    // ---- calcium subsystem and ion concentrations: rates at (V^k, u^k) ----
    const double cai = y[CAI], casr = y[CASR], cass = y[CASS], rbar = y[RBAR];
    double kcasr = MAX_SR - (MAX_SR - MIN_SR) / (1.0 + sq(EC_SR / casr));
    double k1 = K1_PRIME / kcasr;
    double k2 = K2_PRIME * kcasr;
    double open_ = k1 * cass * cass * rbar / (K3 + k1 * cass * cass);
    double i_rel = V_REL * open_ * (casr - cass);
    double i_up = VMAX_UP / (1.0 + sq(K_UP) / sq(cai));
    double i_leak = V_LEAK * (casr - cai);
    double i_xfer = V_XFER * (cass - cai);
    double buf_c = 1.0 / (1.0 + BUF_C * KBUF_C / sq(cai + KBUF_C));
    double buf_sr = 1.0 / (1.0 + BUF_SR * KBUF_SR / sq(casr + KBUF_SR));
    double buf_ss = 1.0 / (1.0 + BUF_SS * KBUF_SS / sq(cass + KBUF_SS));
    double d_rbar = -k2 * cass * rbar + K4 * (1.0 - rbar);
    double d_cai = buf_c * ((i_leak - i_up) * VOLSR / VOLC + i_xfer
                            - (c.ibCa + c.ipCa - 2.0 * c.iNaCa) * CAPAC / (2.0 * VOLC * Far));
    double d_casr = buf_sr * (i_up - i_rel - i_leak);
    double d_cass = buf_ss * (-c.iCaL * CAPAC / (2.0 * VOLSS * Far) + i_rel * VOLSR / VOLSS
                              - i_xfer * VOLC / VOLSS);
    double d_nai = -(c.iNa + c.ibNa + 3.0 * c.iNaK + 3.0 * c.iNaCa) * CAPAC / (VOLC * Far);
    double d_ki = -(c.iK1 + c.ito + c.iKr + c.iKs - 2.0 * c.iNaK + c.ipK) * CAPAC / (VOLC * Far);

    // ---- gating variables at V^k ----
    // fast sodium m, h, j
    double m_inf = 1.0 / sq(1.0 + exp((-56.86 - V) / 9.03));
    double tau_m = (1.0 / (1.0 + exp((-60.0 - V) / 5.0)))
                 * (0.1 / (1.0 + exp((V + 35.0) / 5.0)) + 0.1 / (1.0 + exp((V - 50.0) / 200.0)));
    double h_inf = 1.0 / sq(1.0 + exp((V + 71.55) / 7.43));
    double alpha_h, beta_h, alpha_j, beta_j;
    if (V < -40.0) {
        alpha_h = 0.057 * exp(-(V + 80.0) / 6.8);
        beta_h = 2.7 * exp(0.079 * V) + 3.1e5 * exp(0.3485 * V);
        alpha_j = (-25428.0 * exp(0.2444 * V) - 6.948e-6 * exp(-0.04391 * V)) * (V + 37.78)
                / (1.0 + exp(0.311 * (V + 79.23)));
        beta_j = 0.02424 * exp(-0.01052 * V) / (1.0 + exp(-0.1378 * (V + 40.14)));
    } else {
        alpha_h = 0.0;
        beta_h = 0.77 / (0.13 * (1.0 + exp(-(V + 10.66) / 11.1)));
        alpha_j = 0.0;
        beta_j = 0.6 * exp(0.057 * V) / (1.0 + exp(-0.1 * (V + 32.0)));
    }
    // rapid and slow delayed rectifiers
    double xr1_inf = 1.0 / (1.0 + exp((-26.0 - V) / 7.0));
    double tau_xr1 = (450.0 / (1.0 + exp((-45.0 - V) / 10.0))) * (6.0 / (1.0 + exp((V + 30.0) / 11.5)));
    double xr2_inf = 1.0 / (1.0 + exp((V + 88.0) / 24.0));
    double tau_xr2 = (3.0 / (1.0 + exp((-60.0 - V) / 20.0))) * (1.12 / (1.0 + exp((V - 60.0) / 20.0)));
    double xs_inf = 1.0 / (1.0 + exp((-5.0 - V) / 14.0));
    double tau_xs = (1400.0 / sqrt(1.0 + exp((5.0 - V) / 6.0))) * (1.0 / (1.0 + exp((V - 35.0) / 15.0)))
                  + 80.0;
    // transient outward r, s (endocardial s)
    double r_inf = 1.0 / (1.0 + exp((20.0 - V) / 6.0));
    double tau_r = 9.5 * exp(-sq(V + 40.0) / 1800.0) + 0.8;
    double s_inf = 1.0 / (1.0 + exp((V + 28.0) / 5.0));
    double tau_s = 1000.0 * exp(-sq(V + 67.0) / 1000.0) + 8.0;
    // L-type calcium d, f, f2, fCass
    double d_inf = 1.0 / (1.0 + exp((-8.0 - V) / 7.5));
    double tau_d = (1.4 / (1.0 + exp((-35.0 - V) / 13.0)) + 0.25) * (1.4 / (1.0 + exp((V + 5.0) / 5.0)))
                 + 1.0 / (1.0 + exp((50.0 - V) / 20.0));
    double f_inf = 1.0 / (1.0 + exp((V + 20.0) / 7.0));
    double tau_f = 1102.5 * exp(-sq(V + 27.0) / 225.0) + 200.0 / (1.0 + exp((13.0 - V) / 10.0))
                 + 180.0 / (1.0 + exp((V + 30.0) / 10.0)) + 20.0;
    double f2_inf = 0.67 / (1.0 + exp((V + 35.0) / 7.0)) + 0.33;
    double tau_f2 = 562.0 * exp(-sq(V + 27.0) / 240.0) + 31.0 / (1.0 + exp((25.0 - V) / 10.0))
                  + 80.0 / (1.0 + exp((V + 30.0) / 10.0));
    double cass_ratio2 = sq(cass / 0.05);
    double fcass_inf = 0.6 / (1.0 + cass_ratio2) + 0.4;
    double tau_fcass = 80.0 / (1.0 + cass_ratio2) + 2.0;

    // ---- advance ----
    y[KI] = y[KI] + dt * d_ki;
    y[NAI] = y[NAI] + dt * d_nai;
    y[CAI] = cai + dt * d_cai;
    y[CASR] = casr + dt * d_casr;
    y[CASS] = cass + dt * d_cass;
    y[RBAR] = rbar + dt * d_rbar;
    y[XR1] = rush_larsen(y[XR1], xr1_inf, tau_xr1, dt);
    y[XR2] = rush_larsen(y[XR2], xr2_inf, tau_xr2, dt);
    y[XS] = rush_larsen(y[XS], xs_inf, tau_xs, dt);
    y[MG] = rush_larsen(y[MG], m_inf, tau_m, dt);
    y[HG] = rush_larsen(y[HG], h_inf, 1.0 / (alpha_h + beta_h), dt);
    y[JG] = rush_larsen(y[JG], h_inf, 1.0 / (alpha_j + beta_j), dt);
    y[DG] = rush_larsen(y[DG], d_inf, tau_d, dt);
    y[FG] = rush_larsen(y[FG], f_inf, tau_f, dt);
    y[F2G] = rush_larsen(y[F2G], f2_inf, tau_f2, dt);
    y[FCASS] = rush_larsen(y[FCASS], fcass_inf, tau_fcass, dt);
    y[SG] = rush_larsen(y[SG], s_inf, tau_s, dt);
    y[RG] = rush_larsen(y[RG], r_inf, tau_r, dt);

    // ---- I_ion(V^k, u^{k+1}) ----
    return tt_currents(P, V, vo, y).total();
}

// ---------------------------------------------------------------------------
template <int KIND>
__global__ __launch_bounds__(256) void k_ionic_step(IonicParams P, int64_t n, int64_t ld, double dt,
                                                    double cm, const double *__restrict__ V,
                                                    double *__restrict__ u,
                                                    const double *__restrict__ istim,
                                                    double *__restrict__ out, int raw)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = V[i];
    double iion = 0.0;
    if constexpr (KIND == MDX_KIND_MS) {
        double h = u[i];
        iion = ms_point(P, dt, v, h);
        u[i] = h;
    } else if constexpr (KIND == MDX_KIND_TT) {
        double y[TT_NS];
#pragma unroll
        for (int s = 0; s < TT_NS; ++s) y[s] = u[s * ld + i];
        iion = tt_point(P, dt, v, y);
#pragma unroll
        for (int s = 0; s < TT_NS; ++s) u[s * ld + i] = y[s];
    }
    if (raw)
        out[i] = iion;
    else
        out[i] = (istim ? istim[i] : 0.0) - cm * iion;
}

template <int KIND>
__global__ __launch_bounds__(256) void k_ionic_init(IonicParams P, int64_t n, int64_t ld,
                                                    double *__restrict__ V,
                                                    double *__restrict__ Vprev,
                                                    double *__restrict__ u)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ld) return;
    bool real = i < n;
    double v0 = 0.0;
    if constexpr (KIND == MDX_KIND_MS) {
        v0 = P.v[5];
        if (u) u[i] = real ? 1.0 : 0.0;
    } else if constexpr (KIND == MDX_KIND_TT) {
        v0 = TT_V_REST;
        if (u)
            for (int s = 0; s < TT_NS; ++s) u[s * ld + i] = real ? TT_U0[s] : 0.0;
    }
    V[i] = real ? v0 : 0.0;
    Vprev[i] = real ? v0 : 0.0;
}

IonicParams pack(int kind, const double *params)
{
    IonicParams p{};
    int np = ionic_nparams(kind);
    for (int i = 0; i < np; ++i) p.v[i] = params[i];
    return p;
}

}  // namespace

int ionic_nstates(int kind) { return kind == 1 ? 1 : kind == 2 ? TT_NS : 0; }
int ionic_nparams(int kind) { return kind == 1 ? MS_NP : kind == 2 ? TT_NP : 0; }

void ionic_defaults(int kind, double *params)
{
    static const double ms[MS_NP] = {0.3, 6.0, 120.0, 150.0, 0.13, -80.0, 100.0};
    static const double tt[TT_NP] = {14.838, 5.405, 0.073, 0.153,  0.392,  3.98e-5,
                                     2.9e-4, 5.92e-4, 0.1238, 0.0146, 2.724, 1000.0};
    if (kind == 1)
        for (int i = 0; i < MS_NP; ++i) params[i] = ms[i];
    if (kind == 2)
        for (int i = 0; i < TT_NP; ++i) params[i] = tt[i];
}

void launch_ionic_init(hipStream_t s, int kind, const double *params, int64_t n, int64_t ld,
                       double *V, double *Vprev, double *u)
{
    IonicParams P = pack(kind, params);
    dim3 grid((unsigned)((ld + 255) / 256)), block(256);
    if (kind == 1)
        hipLaunchKernelGGL(k_ionic_init<MDX_KIND_MS>, grid, block, 0, s, P, n, ld, V, Vprev, u);
    else if (kind == 2)
        hipLaunchKernelGGL(k_ionic_init<MDX_KIND_TT>, grid, block, 0, s, P, n, ld, V, Vprev, u);
    else
        hipLaunchKernelGGL(k_ionic_init<MDX_KIND_NONE>, grid, block, 0, s, P, n, ld, V, Vprev, u);
}

void launch_ionic_step(hipStream_t s, int kind, const double *params, int64_t n, int64_t ld,
                       double dt, double cm, const double *V, double *u, const double *istim,
                       double *out, int raw)
{
    if (n <= 0) return;
    IonicParams P = pack(kind, params);
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (kind == 1)
        hipLaunchKernelGGL(k_ionic_step<MDX_KIND_MS>, grid, block, 0, s, P, n, ld, dt, cm, V, u,
                           istim, out, raw);
    else if (kind == 2)
        hipLaunchKernelGGL(k_ionic_step<MDX_KIND_TT>, grid, block, 0, s, P, n, ld, dt, cm, V, u,
                           istim, out, raw);
    else
        hipLaunchKernelGGL(k_ionic_step<MDX_KIND_NONE>, grid, block, 0, s, P, n, ld, dt, cm, V, u,
                           istim, out, raw);
}

}  // namespace mdx
