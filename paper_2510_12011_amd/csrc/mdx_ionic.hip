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

// exponential in the gate precision
__device__ __forceinline__ double ex(double x) { return exp(x); }
__device__ __forceinline__ float ex(float x) { return expf(x); }
__device__ __forceinline__ double sqr_root(double x) { return sqrt(x); }
__device__ __forceinline__ float sqr_root(float x) { return sqrtf(x); }

// Rush-Larsen step y <- y_inf + (y - y_inf) exp(-dt/tau).  In FP32 it is
// evaluated as y + (y_inf - y) (1 - exp(-dt/tau)) with expm1: exp(-dt/tau)
// is within 1e-4 of 1, and rounding it to FP32 would misstate the decay
// rate by ~1e-3, an error that accumulates step after step.
__device__ __forceinline__ double rush_larsen(double y, double y_inf, double tau, double dt)
{
    return y_inf - (y_inf - y) * exp(-dt / tau);
}
__device__ __forceinline__ float rush_larsen(float y, float y_inf, float tau, float dt)
{
    return y - (y_inf - y) * expm1f(-dt / tau);
}
// the same step given the rate 1/tau
__device__ __forceinline__ double rush_larsen_rate(double y, double y_inf, double rate, double dt)
{
    return y_inf - (y_inf - y) * exp(-dt * rate);
}
__device__ __forceinline__ float rush_larsen_rate(float y, float y_inf, float rate, float dt)
{
    return y - (y_inf - y) * expm1f(-dt * rate);
}

// ---------------------------------------------------------------------------
// Mitchell-Schaeffer: params tau_in, tau_out, tau_open, tau_close, u_gate,
// v_rest, v_amp.  dh/dt = (1-h)/tau_open below u_gate, -h/tau_close above;
// I_ion/Cm = -v_amp (h u^2 (1-u)/tau_in - u/tau_out).
// ---------------------------------------------------------------------------
template <typename G>
__device__ __forceinline__ double ms_point(const IonicParams &P, double dt, double V, G &h)
{
    const double tau_in = P.v[0], tau_out = P.v[1], tau_open = P.v[2], tau_close = P.v[3];
    const double u_gate = P.v[4], v_rest = P.v[5], v_amp = P.v[6];
    double u = (V - v_rest) / v_amp;
    bool recovering = u < u_gate;
    G h_inf = recovering ? G(1) : G(0);
    G tau = (G)(recovering ? tau_open : tau_close);
    h = rush_larsen(h, h_inf, tau, (G)dt);
    return -v_amp * ((double)h * u * u * (1.0 - u) / tau_in - u / tau_out);
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
    double w = (V - 15.0) * (2.0 / RTONF);
    o.ical_ew = exp(w);
    o.ical_drive = 2.0 * Far * (w == 0.0 ? 1.0 : w / expm1(w));
    double phi = V * (1.0 / RTONF);
    o.nak_den = 1.0 + 0.1245 * exp(-0.1 * phi) + 0.0353 * exp(-phi);
    o.ncx_up = exp(NCX_GAMMA * phi);
    o.ncx_down = exp((NCX_GAMMA - 1.0) * phi);
    o.ncx_sat = 1.0 + K_SAT * o.ncx_down;
    o.ipk = 1.0 / (1.0 + exp((25.0 - V) * (1.0 / 5.98)));
    return o;
}

// Products of the gating variables that enter the currents, formed in FP64
// from the stored gates: the currents need these five numbers, not the
// twelve gates, which keeps the live set of a thread small.
struct GateProducts {
    double to;    // r s           (transient outward)
    double kr;    // xr1 xr2       (rapid delayed rectifier)
    double ks;    // xs^2          (slow delayed rectifier)
    double na;    // m^3 h j       (fast sodium)
    double cal;   // d f f2 fCass  (L-type calcium)
};

struct Currents {
    double iK1, ito, iKr, iKs, iCaL, iNaK, iNa, ibNa, iNaCa, ibCa, ipK, ipCa;
    __device__ double total() const
    {
        return iK1 + ito + iKr + iKs + iCaL + iNaK + iNa + ibNa + iNaCa + ibCa + ipK + ipCa;
    }
};

// currents at V and the concentration-type states c[0..5] (Ki Nai Cai CaSR
// CaSS Rbar) and gates summarised by gp
__device__ __forceinline__ Currents tt_currents(const IonicParams &P, double V, const VOnly &vo,
                                                const double *c, const GateProducts &gp)
{
    const double gNa = P.v[0], gK1 = P.v[1], gto = P.v[2], gKr = P.v[3], gKs = P.v[4];
    const double gCaL = P.v[5], gbNa = P.v[6], gbCa = P.v[7], gpCa = P.v[8], gpK = P.v[9];
    const double pNaK = P.v[10], kNaCa = P.v[11];
    const double ki = c[KI], nai = c[NAI], cai = c[CAI];
    const double e_k = RTONF * log(K_O / ki);
    const double e_na = RTONF * log(NA_O / nai);
    const double e_ks = RTONF * log((K_O + P_KNA * NA_O) / (ki + P_KNA * nai));
    const double e_ca = 0.5 * RTONF * log(CA_O / cai);
    const double ko_scale = sqrt(K_O / 5.4);
    Currents cu;
    // inward rectifier: steady-state rectification a/(a+b) with
    // a = 0.1/(1+e1), b = q/(1+e2), formed as 0.1(1+e2) / (0.1(1+e2) + q(1+e1))
    const double a_k1 = 0.1 * (1.0 + exp(-0.5 * (V - e_k)));
    const double b_k1 = (3.0 * exp(0.0002 * (V - e_k + 100.0)) + exp(0.1 * (V - e_k - 10.0)))
                      * (1.0 + exp(0.06 * (V - e_k - 200.0)));
    cu.iK1 = gK1 * ko_scale * (a_k1 / (a_k1 + b_k1)) * (V - e_k);
    cu.ito = gto * gp.to * (V - e_k);
    cu.iKr = gKr * ko_scale * gp.kr * (V - e_k);
    cu.iKs = gKs * gp.ks * (V - e_ks);
    cu.iNa = gNa * gp.na * (V - e_na);
    cu.ibNa = gbNa * (V - e_na);
    cu.iCaL = gCaL * gp.cal * vo.ical_drive * (0.25 * c[CASS] * vo.ical_ew - CA_O);
    cu.ibCa = gbCa * (V - e_ca);
    cu.iNaK = pNaK * (K_O / (K_O + KM_K)) * nai / ((nai + KM_NA) * vo.nak_den);
    constexpr double nao3 = NA_O * NA_O * NA_O;
    constexpr double ncx_den = (KM_NAI * KM_NAI * KM_NAI + nao3) * (KM_CA + CA_O);
    cu.iNaCa = kNaCa * (vo.ncx_up * nai * nai * nai * CA_O - vo.ncx_down * nao3 * cai * NCX_ALPHA)
             / (ncx_den * vo.ncx_sat);
    cu.ipCa = gpCa * cai / (K_PCA + cai);
    cu.ipK = gpK * vo.ipk * (V - e_k);
    return cu;
}

__device__ __forceinline__ double sq(double x) { return x * x; }

// Gating variables of the model advanced by Rush-Larsen at V^k, in precision
// T, streamed one at a time: gate s (xr1 xr2 xs m h j d f f2 fCass s r) is
// read from g[s * ld], advanced and written back at once.  po and pn receive
// the gate products before and after the step; cass is CaSS^k.
template <typename T>
__device__ __forceinline__ void tt_gates(T V, T dt, T cass, T *__restrict__ g, int64_t ld,
                                         GateProducts &po, GateProducts &pn)
{
    const T one = T(1);
    auto sqt = [](T x) { return x * x; };
    // advance gate s towards y_inf with time constant tau; old value to y0
    auto adv = [&](int s, T y_inf, T tau, double &y0) -> double {
        const T y = g[s * ld];
        const T y1 = rush_larsen(y, y_inf, tau, dt);
        g[s * ld] = y1;
        y0 = (double)y;
        return (double)y1;
    };
    auto adv_rate = [&](int s, T y_inf, T rate, double &y0) -> double {
        const T y = g[s * ld];
        const T y1 = rush_larsen_rate(y, y_inf, rate, dt);
        g[s * ld] = y1;
        y0 = (double)y;
        return (double)y1;
    };
    double o0, o1, o2, n0, n1, n2;

    // rapid delayed rectifier xr1, xr2
    {
        T inf = one / (one + ex((T(-26.0) - V) * T(1.0 / 7.0)));
        // 450/(1+a) * 6/(1+b) with one division
        T tau = T(450.0 * 6.0) / ((one + ex((T(-45.0) - V) * T(1.0 / 10.0))) * (one + ex((V + T(30.0)) * T(1.0 / 11.5))));
        n0 = adv(0, inf, tau, o0);
    }
    {
        T inf = one / (one + ex((V + T(88.0)) * T(1.0 / 24.0)));
        T tau = T(3.0 * 1.12) / ((one + ex((T(-60.0) - V) * T(1.0 / 20.0))) * (one + ex((V - T(60.0)) * T(1.0 / 20.0))));
        n1 = adv(1, inf, tau, o1);
    }
    po.kr = o0 * o1;
    pn.kr = n0 * n1;
    // slow delayed rectifier xs
    {
        T inf = one / (one + ex((T(-5.0) - V) * T(1.0 / 14.0)));
        T tau = T(1400.0) / (sqr_root(one + ex((T(5.0) - V) * T(1.0 / 6.0))) * (one + ex((V - T(35.0)) * T(1.0 / 15.0))))
              + T(80.0);
        n0 = adv(2, inf, tau, o0);
    }
    po.ks = o0 * o0;
    pn.ks = n0 * n0;
    // fast sodium m, h, j
    {
        T inf = one / sqt(one + ex((T(-56.86) - V) * T(1.0 / 9.03)));
        T tau = (one / (one + ex((T(-60.0) - V) * T(1.0 / 5.0))))
              * (T(0.1) / (one + ex((V + T(35.0)) * T(1.0 / 5.0))) + T(0.1) / (one + ex((V - T(50.0)) * T(1.0 / 200.0))));
        n0 = adv(3, inf, tau, o0);
    }
    {
        T h_inf = one / sqt(one + ex((V + T(71.55)) * T(1.0 / 7.43)));
        T alpha_h, beta_h, alpha_j, beta_j;
        if (V < T(-40.0)) {
            alpha_h = T(0.057) * ex(-(V + T(80.0)) * T(1.0 / 6.8));
            beta_h = T(2.7) * ex(T(0.079) * V) + T(3.1e5) * ex(T(0.3485) * V);
            alpha_j = (T(-25428.0) * ex(T(0.2444) * V) - T(6.948e-6) * ex(T(-0.04391) * V)) * (V + T(37.78))
                    / (one + ex(T(0.311) * (V + T(79.23))));
            beta_j = T(0.02424) * ex(T(-0.01052) * V) / (one + ex(T(-0.1378) * (V + T(40.14))));
        } else {
            alpha_h = T(0.0);
            beta_h = T(0.77 / 0.13) / (one + ex(-(V + T(10.66)) * T(1.0 / 11.1)));
            alpha_j = T(0.0);
            beta_j = T(0.6) * ex(T(0.057) * V) / (one + ex(T(-0.1) * (V + T(32.0))));
        }
        n1 = adv_rate(4, h_inf, alpha_h + beta_h, o1);
        n2 = adv_rate(5, h_inf, alpha_j + beta_j, o2);
    }
    po.na = o0 * o0 * o0 * o1 * o2;
    pn.na = n0 * n0 * n0 * n1 * n2;
    // L-type calcium d, f, f2, fCass
    {
        T inf = one / (one + ex((T(-8.0) - V) * T(1.0 / 7.5)));
        T tau = (T(1.4) / (one + ex((T(-35.0) - V) * T(1.0 / 13.0))) + T(0.25)) * (T(1.4) / (one + ex((V + T(5.0)) * T(1.0 / 5.0))))
              + one / (one + ex((T(50.0) - V) * T(1.0 / 20.0)));
        n0 = adv(6, inf, tau, o0);
    }
    {
        T inf = one / (one + ex((V + T(20.0)) * T(1.0 / 7.0)));
        T tau = T(1102.5) * ex(-sqt(V + T(27.0)) * T(1.0 / 225.0)) + T(200.0) / (one + ex((T(13.0) - V) * T(1.0 / 10.0)))
              + T(180.0) / (one + ex((V + T(30.0)) * T(1.0 / 10.0))) + T(20.0);
        n1 = adv(7, inf, tau, o1);
    }
    po.cal = o0 * o1;
    pn.cal = n0 * n1;
    {
        T inf = T(0.67) / (one + ex((V + T(35.0)) * T(1.0 / 7.0))) + T(0.33);
        T tau = T(562.0) * ex(-sqt(V + T(27.0)) * T(1.0 / 240.0)) + T(31.0) / (one + ex((T(25.0) - V) * T(1.0 / 10.0)))
              + T(80.0) / (one + ex((V + T(30.0)) * T(1.0 / 10.0)));
        n0 = adv(8, inf, tau, o0);
    }
    {
        T ratio2 = sqt(cass * T(1.0 / 0.05));
        T inf = T(0.6) / (one + ratio2) + T(0.4);
        T tau = T(80.0) / (one + ratio2) + T(2.0);
        n1 = adv(9, inf, tau, o1);
    }
    po.cal = po.cal * o0 * o1;
    pn.cal = pn.cal * n0 * n1;
    // transient outward s (endocardial), r
    {
        T inf = one / (one + ex((V + T(28.0)) * T(1.0 / 5.0)));
        T tau = T(1000.0) * ex(-sqt(V + T(67.0)) * T(1.0 / 1000.0)) + T(8.0);
        n0 = adv(10, inf, tau, o0);
    }
    {
        T inf = one / (one + ex((T(20.0) - V) * T(1.0 / 6.0)));
        T tau = T(9.5) * ex(-sqt(V + T(40.0)) * T(1.0 / 1800.0)) + T(0.8);
        n1 = adv(11, inf, tau, o1);
    }
    po.to = o1 * o0;
    pn.to = n1 * n0;
}

// One step of the model at one node: concentration-type states c[0..5]
// (Ki Nai Cai CaSR CaSS Rbar) by forward Euler in FP64, gates (g[s * ld],
// s = 0..11) by Rush-Larsen in precision G; returns I_ion(V^k, u^{k+1}) / Cm
// in FP64.
template <typename G>
__device__ double tt_point(const IonicParams &P, double dt, double V, double *c,
                           G *__restrict__ g, int64_t ld)
{
    const VOnly vo = v_only(V);
    const double cai = c[CAI], casr = c[CASR], cass = c[CASS], rbar = c[RBAR];

    // ---- gating variables at V^k (their products at u^k and u^{k+1}) ----
    GateProducts po, pn;
    tt_gates<G>((G)V, (G)dt, (G)cass, g, ld, po, pn);

    // ---- calcium subsystem and ion concentrations: rates at (V^k, u^k) ----
    const Currents cur = tt_currents(P, V, vo, c, po);
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
    double d_cai = buf_c * ((i_leak - i_up) * (VOLSR / VOLC) + i_xfer
                            - (cur.ibCa + cur.ipCa - 2.0 * cur.iNaCa) * (CAPAC / (2.0 * VOLC * Far)));
    double d_casr = buf_sr * (i_up - i_rel - i_leak);
    double d_cass = buf_ss * (-cur.iCaL * (CAPAC / (2.0 * VOLSS * Far)) + i_rel * (VOLSR / VOLSS)
                              - i_xfer * (VOLC / VOLSS));
    double d_nai = -(cur.iNa + cur.ibNa + 3.0 * cur.iNaK + 3.0 * cur.iNaCa) * (CAPAC / (VOLC * Far));
    double d_ki = -(cur.iK1 + cur.ito + cur.iKr + cur.iKs - 2.0 * cur.iNaK + cur.ipK) * (CAPAC / (VOLC * Far));

    // ---- forward Euler for the concentration-type states ----
    c[KI] = c[KI] + dt * d_ki;
    c[NAI] = c[NAI] + dt * d_nai;
    c[CAI] = cai + dt * d_cai;
    c[CASR] = casr + dt * d_casr;
    c[CASS] = cass + dt * d_cass;
    c[RBAR] = rbar + dt * d_rbar;

    // ---- I_ion(V^k, u^{k+1}) ----
    return tt_currents(P, V, vo, c, pn).total();
}

// Row i holds a cell: i < n, or, with the per-tile count of real rows of the
// batched layout (padding rows at the end of each instance's last tile),
// (i mod TILE) < tile_real[i / TILE].
__device__ __forceinline__ bool real_row(int64_t i, int64_t n, const int32_t *tile_real)
{
    return tile_real ? (int)(i & (TILE - 1)) < tile_real[i / TILE] : i < n;
}

// ---------------------------------------------------------------------------
// The ten Tusscher-Panfilov update is latency bound (a chain of FP64
// exponentials per node); streaming the gates through tt_gates keeps it at
// ~123 registers, four wavefronts per SIMD with no spills.  A tighter bound
// spills more than it gains.
template <int KIND>
__global__ __launch_bounds__(256) void k_ionic_step(IonicParams P, int64_t n, int64_t ld, double dt,
                                                    double cm, const double *__restrict__ V,
                                                    double *__restrict__ u,
                                                    const double *__restrict__ istim,
                                                    double *__restrict__ out, int raw,
                                                    const int32_t *__restrict__ tile_real,
                                                    const int32_t *__restrict__ guard)
{
    if (guard && !*guard) return;   // enqueued ahead of a solve that is not done
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!real_row(i, n, tile_real)) {
        out[i] = 0.0;
        return;
    }
    double v = V[i];
    double iion = 0.0;
    if constexpr (KIND == MDX_KIND_MS) {
        double h = u[i];
        iion = ms_point<double>(P, dt, v, h);
        u[i] = h;
    } else if constexpr (KIND == MDX_KIND_TT) {
        double c[6];
#pragma unroll
        for (int s = 0; s < 6; ++s) c[s] = u[s * ld + i];
        iion = tt_point<double>(P, dt, v, c, u + 6 * ld + i, ld);
#pragma unroll
        for (int s = 0; s < 6; ++s) u[s * ld + i] = c[s];
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
                                                    double *__restrict__ u,
                                                    const int32_t *__restrict__ tile_real)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ld) return;
    const bool real = real_row(i, n, tile_real);
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

// Mixed-precision form: gating variables stored and advanced in FP32
// (g32[s * ld + i], s over the model's gates), concentration-type states and
// the current in FP64 (u[s * ld + i], rows 0..5 for the ten Tusscher-Panfilov
// model; Mitchell-Schaeffer has only its gate h).
template <int KIND>
__global__ __launch_bounds__(256) void k_ionic_step_mixed(IonicParams P, int64_t n, int64_t ld,
                                                          double dt, double cm,
                                                          const double *__restrict__ V,
                                                          double *__restrict__ u,
                                                          float *__restrict__ g32,
                                                          const double *__restrict__ istim,
                                                          double *__restrict__ out,
                                                          const int32_t *__restrict__ tile_real,
                                                          const int32_t *__restrict__ guard)
{
    if (guard && !*guard) return;   // enqueued ahead of a solve that is not done
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!real_row(i, n, tile_real)) {
        out[i] = 0.0;
        return;
    }
    const double v = V[i];
    double iion = 0.0;
    if constexpr (KIND == MDX_KIND_MS) {
        float h = g32[i];
        iion = ms_point<float>(P, dt, v, h);
        g32[i] = h;
    } else if constexpr (KIND == MDX_KIND_TT) {
        double c[6];
#pragma unroll
        for (int s = 0; s < 6; ++s) c[s] = u[s * ld + i];
        iion = tt_point<float>(P, dt, v, c, g32 + i, ld);
#pragma unroll
        for (int s = 0; s < 6; ++s) u[s * ld + i] = c[s];
    }
    out[i] = (istim ? istim[i] : 0.0) - cm * iion;
}

// copy rows [row0, row0 + rows) of an FP64 SoA state block to FP32 or back
__global__ __launch_bounds__(256) void k_rows_to_f32(int64_t ld, int rows, const double *__restrict__ src,
                                                     float *__restrict__ dst)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ld * rows) return;
    dst[i] = (float)src[i];
}

__global__ __launch_bounds__(256) void k_rows_to_f64(int64_t ld, int rows, const float *__restrict__ src,
                                                     double *__restrict__ dst)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ld * rows) return;
    dst[i] = (double)src[i];
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
                       double *V, double *Vprev, double *u, const int32_t *tile_real)
{
    IonicParams P = pack(kind, params);
    dim3 grid((unsigned)((ld + 255) / 256)), block(256);
    if (kind == 1)
        hipLaunchKernelGGL(k_ionic_init<MDX_KIND_MS>, grid, block, 0, s, P, n, ld, V, Vprev, u, tile_real);
    else if (kind == 2)
        hipLaunchKernelGGL(k_ionic_init<MDX_KIND_TT>, grid, block, 0, s, P, n, ld, V, Vprev, u, tile_real);
    else
        hipLaunchKernelGGL(k_ionic_init<MDX_KIND_NONE>, grid, block, 0, s, P, n, ld, V, Vprev, u, tile_real);
}

void launch_ionic_step(hipStream_t s, int kind, const double *params, int64_t n, int64_t ld,
                       double dt, double cm, const double *V, double *u, const double *istim,
                       double *out, int raw, const int32_t *tile_real, const int32_t *guard)
{
    if (n <= 0) return;
    IonicParams P = pack(kind, params);
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (kind == 1)
        hipLaunchKernelGGL(k_ionic_step<MDX_KIND_MS>, grid, block, 0, s, P, n, ld, dt, cm, V, u,
                           istim, out, raw, tile_real, guard);
    else if (kind == 2)
        hipLaunchKernelGGL(k_ionic_step<MDX_KIND_TT>, grid, block, 0, s, P, n, ld, dt, cm, V, u,
                           istim, out, raw, tile_real, guard);
    else
        hipLaunchKernelGGL(k_ionic_step<MDX_KIND_NONE>, grid, block, 0, s, P, n, ld, dt, cm, V, u,
                           istim, out, raw, tile_real, guard);
}

int ionic_gate_rows(int kind) { return kind == 1 ? 1 : kind == 2 ? 12 : 0; }
int ionic_gate_row0(int kind) { return kind == 1 ? 0 : kind == 2 ? 6 : 0; }

void launch_ionic_step_mixed(hipStream_t s, int kind, const double *params, int64_t n, int64_t ld,
                             double dt, double cm, const double *V, double *u, float *g32,
                             const double *istim, double *out, const int32_t *tile_real,
                             const int32_t *guard)
{
    if (n <= 0) return;
    IonicParams P = pack(kind, params);
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (kind == 1)
        hipLaunchKernelGGL(k_ionic_step_mixed<MDX_KIND_MS>, grid, block, 0, s, P, n, ld, dt, cm, V,
                           u, g32, istim, out, tile_real, guard);
    else if (kind == 2)
        hipLaunchKernelGGL(k_ionic_step_mixed<MDX_KIND_TT>, grid, block, 0, s, P, n, ld, dt, cm, V,
                           u, g32, istim, out, tile_real, guard);
    else
        hipLaunchKernelGGL(k_ionic_step_mixed<MDX_KIND_NONE>, grid, block, 0, s, P, n, ld, dt, cm,
                           V, u, g32, istim, out, tile_real, guard);
}

void launch_gates_to_f32(hipStream_t s, int kind, int64_t ld, const double *u, float *g32)
{
    const int rows = ionic_gate_rows(kind);
    if (rows == 0) return;
    const int64_t cnt = ld * rows;
    hipLaunchKernelGGL(k_rows_to_f32, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, ld, rows,
                       u + (int64_t)ionic_gate_row0(kind) * ld, g32);
}

void launch_gates_to_f64(hipStream_t s, int kind, int64_t ld, const float *g32, double *u)
{
    const int rows = ionic_gate_rows(kind);
    if (rows == 0) return;
    const int64_t cnt = ld * rows;
    hipLaunchKernelGGL(k_rows_to_f64, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, ld, rows,
                       g32, u + (int64_t)ionic_gate_row0(kind) * ld);
}

}  // namespace mdx
