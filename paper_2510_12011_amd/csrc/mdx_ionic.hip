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
//    (Am. J. Physiol. Heart Circ. Physiol. 291:H1088), 18 states + V;
//  * Courtemanche-Ramirez-Nattel 1998 human atrial model (Am. J. Physiol.
//    275:H301), 20 states + V.
#include "mdx_device.h"
#include "mdx_internal.h"

namespace mdx {

namespace {

enum { MDX_KIND_NONE = 0, MDX_KIND_MS = 1, MDX_KIND_TT = 2, MDX_KIND_CRN = 3 };
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

// ---------------------------------------------------------------------------
// Courtemanche-Ramirez-Nattel 1998 human atrial cell (Am. J. Physiol. 275:
// H301), 20 states + V, held in registers for the step:
//   y[0..4]  Na_i K_i Ca_i Ca_up Ca_rel (mM; forward Euler)
//   y[5..19] m h j oa oi ua ui xr xs d f fCa u v w (Rush-Larsen)
// params: gNa gK1 gto gKr gKs gCaL gbNa gbCa (nS/pF), INaK_max INaCa_max
// IpCa_max (pA/pF), Iup_max (mM/ms), and a scale of gKur(V).
// Currents are per unit capacitance; the membrane capacitance (100 pF) turns
// them into the pA that the concentration balances and the release trigger
// use.
// ---------------------------------------------------------------------------
namespace crn {
constexpr double RT_F = 8.3143 * 310.0 / 96.4867;   // mV
constexpr double FARADAY = 96.4867;                   // C/mmol
constexpr double CAP = 100.0;                         // pF
constexpr double VOL_I = 13668.0, VOL_UP = 1109.52, VOL_REL = 96.48;   // um^3
constexpr double K_OUT = 5.4, NA_OUT = 140.0, CA_OUT = 1.8;
constexpr double NAK_KM_NA = 10.0, NAK_KM_K = 1.5;
constexpr double NACA_KM_NA = 87.5, NACA_KM_CA = 1.38, NACA_SAT = 0.1, NACA_GAMMA = 0.35;
constexpr double REL_RATE = 30.0, UP_KM = 0.00092, UP_CA_MAX = 15.0, TR_TAU = 180.0;
constexpr double CMDN_TOT = 0.05, CMDN_KM = 0.00238, TRPN_TOT = 0.07, TRPN_KM = 0.0005;
constexpr double CSQN_TOT = 10.0, CSQN_KM = 0.8;
constexpr double Q10 = 3.0;
constexpr double V_REST = -81.18;
// ratio of the sodium-potassium pump's [Na]_o dependence, (e^{Na_o/67.3} - 1) / 7
__device__ __forceinline__ double nak_sigma() { return (exp(NA_OUT / 67.3) - 1.0) / 7.0; }
}  // namespace crn
constexpr int CRN_NS = 20;
constexpr int CRN_NP = 13;
__device__ const double CRN_U0[CRN_NS] = {11.17,  139.0,  1.013e-4, 1.488,    1.488,
                                          2.908e-3, 0.9649, 0.9775, 3.043e-2, 0.9992,
                                          4.966e-3, 0.9986, 3.296e-5, 1.869e-2, 1.367e-4,
                                          0.9996, 0.7755, 0.0,      1.0,      0.9992};

// x / (1 - e^{-x/s}), whose limit at x = 0 is s
__device__ __forceinline__ double rise_ratio(double x, double s)
{
    const double t = x / s;
    return t != 0.0 ? x / -expm1(-t) : s;
}
// x / (e^{x/s} - 1), whose limit at x = 0 is s
__device__ __forceinline__ double fall_ratio(double x, double s)
{
    const double t = x / s;
    return t != 0.0 ? x / expm1(t) : s;
}
__device__ __forceinline__ double logistic(double x) { return 1.0 / (1.0 + exp(-x)); }

struct CrnCurrents {
    double iNa, iK1, ito, iKur, iKr, iKs, iCaL, iNaK, iNaCa, ibNa, ibCa, ipCa;
    __device__ double total() const
    {
        return ((iNa + ibNa) + (iK1 + ito + iKur + iKr + iKs)) + ((iCaL + ibCa + ipCa) + (iNaK + iNaCa));
    }
};

__device__ __forceinline__ CrnCurrents crn_currents(const IonicParams &P, double V, const double *y)
{
    using namespace crn;
    const double na = y[0], k = y[1], ca = y[2];
    const double e_na = RT_F * log(NA_OUT / na), e_k = RT_F * log(K_OUT / k);
    const double e_ca = 0.5 * RT_F * log(CA_OUT / ca);
    const double u = V * (1.0 / RT_F);
    CrnCurrents c;
    const double m = y[5];
    c.iNa = P.v[0] * (m * m * m) * y[6] * y[7] * (V - e_na);
    c.iK1 = P.v[1] * (V - e_k) * logistic(-0.07 * (V + 80.0));
    const double oa = y[8];
    c.ito = P.v[2] * (oa * oa * oa) * y[9] * (V - e_k);
    const double ua = y[10];
    const double g_kur = P.v[12] * (0.005 + 0.05 * logistic((V - 15.0) * (1.0 / 13.0)));
    c.iKur = g_kur * (ua * ua * ua) * y[11] * (V - e_k);
    c.iKr = P.v[3] * y[12] * (V - e_k) * logistic(-(V + 15.0) * (1.0 / 22.4));
    c.iKs = P.v[4] * y[13] * y[13] * (V - e_k);
    c.iCaL = P.v[5] * y[14] * y[15] * y[16] * (V - 65.0);
    const double pump_v = 1.0 / (1.0 + 0.1245 * exp(-0.1 * u) + 0.0365 * nak_sigma() * exp(-u));
    const double pump_na = 1.0 / (1.0 + (NAK_KM_NA / na) * sqrt(NAK_KM_NA / na));
    c.iNaK = P.v[8] * pump_v * pump_na * (K_OUT / (K_OUT + NAK_KM_K));
    const double e_in = exp(NACA_GAMMA * u), e_out = exp((NACA_GAMMA - 1.0) * u);
    const double km3 = NACA_KM_NA * NACA_KM_NA * NACA_KM_NA, nao3 = NA_OUT * NA_OUT * NA_OUT;
    c.iNaCa = P.v[9] * (e_in * (na * na * na) * CA_OUT - e_out * nao3 * ca)
            / ((km3 + nao3) * (NACA_KM_CA + CA_OUT) * (1.0 + NACA_SAT * e_out));
    c.ibNa = P.v[6] * (V - e_na);
    c.ibCa = P.v[7] * (V - e_ca);
    c.ipCa = P.v[10] * ca / (0.0005 + ca);
    return c;
}

// One step at one node: fluxes and rates at (V^k, u^k), then u^{k+1};
// returns I_ion(V^k, u^{k+1}) / Cm (mV/ms).
__device__ double crn_point(const IonicParams &P, double dt, double V, double *y)
{
    using namespace crn;
    const CrnCurrents c = crn_currents(P, V, y);
    const double ca = y[2], ca_up = y[3], ca_rel = y[4];
    const double uu = y[17];
    const double j_rel = REL_RATE * (uu * uu) * y[18] * y[19] * (ca_rel - ca);
    const double j_tr = (ca_up - ca_rel) * (1.0 / TR_TAU);
    const double j_up = P.v[11] / (1.0 + UP_KM / ca);
    const double j_leak = P.v[11] * ca_up * (1.0 / UP_CA_MAX);
    // current (pA/pF) to concentration rate in the myoplasm (mM/ms)
    constexpr double to_conc = CAP / (FARADAY * VOL_I);
    const double d_na = -to_conc * (3.0 * (c.iNaK + c.iNaCa) + c.ibNa + c.iNa);
    const double d_k = to_conc * (2.0 * c.iNaK - (c.iK1 + c.ito + c.iKur + c.iKr + c.iKs));
    const double free_ca = 0.5 * to_conc * (2.0 * c.iNaCa - c.ipCa - c.iCaL - c.ibCa)
                         + (VOL_UP * (j_leak - j_up) + VOL_REL * j_rel) * (1.0 / VOL_I);
    const double b_cmdn = CMDN_TOT * CMDN_KM / ((ca + CMDN_KM) * (ca + CMDN_KM));
    const double b_trpn = TRPN_TOT * TRPN_KM / ((ca + TRPN_KM) * (ca + TRPN_KM));
    const double d_ca = free_ca / (1.0 + b_trpn + b_cmdn);
    const double d_up = j_up - j_leak - j_tr * (VOL_REL / VOL_UP);
    const double d_rel = (j_tr - j_rel) / (1.0 + CSQN_TOT * CSQN_KM / ((ca_rel + CSQN_KM) * (ca_rel + CSQN_KM)));

    // release trigger: SR release plus the Ca entry of I_CaL and I_NaCa (pA)
    const double fn = 1e-12 * VOL_REL * j_rel - (5e-13 / FARADAY) * CAP * (0.5 * c.iCaL - 0.2 * c.iNaCa);
    const double on_u = logistic((fn - 3.4175e-13) * (1.0 / 13.67e-16));

    // ---- gates: Rush-Larsen with the rate 1/tau at V^k ----
    {   // fast sodium m, h, j from their opening and closing rates
        const double am = 0.32 * rise_ratio(V + 47.13, 10.0), bm = 0.08 * exp(-V * (1.0 / 11.0));
        y[5] = rush_larsen_rate(y[5], am / (am + bm), am + bm, dt);
        double ah = 0.0, bh, aj = 0.0, bj;
        if (V < -40.0) {
            ah = 0.135 * exp(-(V + 80.0) * (1.0 / 6.8));
            bh = 3.56 * exp(0.079 * V) + 3.1e5 * exp(0.35 * V);
            aj = (-127140.0 * exp(0.2444 * V) - 3.474e-5 * exp(-0.04391 * V)) * (V + 37.78)
               * logistic(-0.311 * (V + 79.23));
            bj = 0.1212 * exp(-0.01052 * V) * logistic(0.1378 * (V + 40.14));
        } else {
            bh = (1.0 / 0.13) * logistic((V + 10.66) * (1.0 / 11.1));
            bj = 0.3 * exp(-2.535e-7 * V) * logistic(0.1 * (V + 32.0));
        }
        y[6] = rush_larsen_rate(y[6], ah / (ah + bh), ah + bh, dt);
        y[7] = rush_larsen_rate(y[7], aj / (aj + bj), aj + bj, dt);
    }
    {   // transient (oa, oi) and ultrarapid (ua, ui) potassium, Q10 = 3
        const double a_a = 0.65 / (exp(-(V + 10.0) * (1.0 / 8.5)) + exp(-(V - 30.0) * (1.0 / 59.0)));
        const double b_a = 0.65 / (2.5 + exp((V + 82.0) * (1.0 / 17.0)));
        const double r_a = (a_a + b_a) * Q10;
        y[8] = rush_larsen_rate(y[8], logistic((V + 20.47) * (1.0 / 17.54)), r_a, dt);
        y[10] = rush_larsen_rate(y[10], logistic((V + 30.3) * (1.0 / 9.6)), r_a, dt);
        const double a_oi = 1.0 / (18.53 + exp((V + 113.7) * (1.0 / 10.95)));
        const double b_oi = 1.0 / (35.56 + exp(-(V + 1.26) * (1.0 / 7.44)));
        y[9] = rush_larsen_rate(y[9], logistic(-(V + 43.1) * (1.0 / 5.3)), (a_oi + b_oi) * Q10, dt);
        const double a_ui = 1.0 / (21.0 + exp(-(V - 185.0) * (1.0 / 28.0)));
        const double b_ui = exp((V - 158.0) * (1.0 / 16.0));
        y[11] = rush_larsen_rate(y[11], logistic(-(V - 99.45) * (1.0 / 27.48)), (a_ui + b_ui) * Q10, dt);
    }
    {   // rapid and slow delayed rectifiers
        const double a_r = 0.0003 * rise_ratio(V + 14.1, 5.0);
        const double b_r = 7.3898e-5 * fall_ratio(V - 3.3328, 5.1237);
        y[12] = rush_larsen_rate(y[12], logistic((V + 14.1) * (1.0 / 6.5)), a_r + b_r, dt);
        const double a_s = 4e-5 * rise_ratio(V - 19.9, 17.0);
        const double b_s = 3.5e-5 * fall_ratio(V - 19.9, 9.0);
        y[13] = rush_larsen_rate(y[13], sqrt(logistic((V - 19.9) * (1.0 / 12.7))), 2.0 * (a_s + b_s), dt);
    }
    {   // L-type calcium d, f, fCa
        const double x = V + 10.0;
        // 1/tau_d = 0.035 x (1 + e^{-x/6.24}) / (1 - e^{-x/6.24})
        const double r_d = 0.035 * rise_ratio(x, 6.24) * (1.0 + exp(-x * (1.0 / 6.24)));
        y[14] = rush_larsen_rate(y[14], logistic(x * (1.0 / 8.0)), r_d, dt);
        const double r_f = (0.0197 * exp(-(0.0337 * 0.0337) * x * x) + 0.02) * (1.0 / 9.0);
        y[15] = rush_larsen_rate(y[15], logistic(-(V + 28.0) * (1.0 / 6.9)), r_f, dt);
        y[16] = rush_larsen_rate(y[16], 1.0 / (1.0 + ca * (1.0 / 0.00035)), 0.5, dt);
    }
    {   // SR release gates u, v (trigger fn) and w (voltage)
        y[17] = rush_larsen_rate(y[17], on_u, 1.0 / 8.0, dt);
        const double v_inf = 1.0 - logistic((fn - 6.835e-14) * (1.0 / 13.67e-16));
        y[18] = rush_larsen_rate(y[18], v_inf, 1.0 / (1.91 + 2.09 * on_u), dt);
        const double xw = V - 7.9;
        // 1/tau_w = x (1 + 0.3 e^{-x/5}) / (6 (1 - e^{-x/5}))
        const double r_w = rise_ratio(xw, 5.0) * (1.0 + 0.3 * exp(-xw * (1.0 / 5.0))) * (1.0 / 6.0);
        y[19] = rush_larsen_rate(y[19], 1.0 - logistic((V - 40.0) * (1.0 / 17.0)), r_w, dt);
    }
    // ---- forward Euler for the concentrations ----
    y[0] += dt * d_na;
    y[1] += dt * d_k;
    y[2] = ca + dt * d_ca;
    y[3] = ca_up + dt * d_up;
    y[4] = ca_rel + dt * d_rel;
    return crn_currents(P, V, y).total();
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
                                                    const int32_t *__restrict__ guard,
                                                    StepTimes times)
{
    if (guard && !*guard) return;   // enqueued ahead of a solve that is not done
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!real_row(i, n, tile_real)) {
        out[i] = 0.0;
        return;
    }
    double v = V[i];
    if (times.lat && !update_times(i, times.t1, times.Vold[i], v, times.lat, times.lrt))
        times.sc->nonfinite_v = 1;
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
    } else if constexpr (KIND == MDX_KIND_CRN) {
        double y[CRN_NS];
#pragma unroll
        for (int s = 0; s < CRN_NS; ++s) y[s] = u[s * ld + i];
        iion = crn_point(P, dt, v, y);
#pragma unroll
        for (int s = 0; s < CRN_NS; ++s) u[s * ld + i] = y[s];
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
    } else if constexpr (KIND == MDX_KIND_CRN) {
        v0 = crn::V_REST;
        // padding rows hold the rest state too (finite logarithms if read)
        if (u)
            for (int s = 0; s < CRN_NS; ++s) u[s * ld + i] = CRN_U0[s];
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
                                                          const int32_t *__restrict__ guard,
                                                          StepTimes times)
{
    if (guard && !*guard) return;   // enqueued ahead of a solve that is not done
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!real_row(i, n, tile_real)) {
        out[i] = 0.0;
        return;
    }
    const double v = V[i];
    if (times.lat && !update_times(i, times.t1, times.Vold[i], v, times.lat, times.lrt))
        times.sc->nonfinite_v = 1;
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

int ionic_nstates(int kind) { return kind == 1 ? 1 : kind == 2 ? TT_NS : kind == 3 ? CRN_NS : 0; }
int ionic_nparams(int kind) { return kind == 1 ? MS_NP : kind == 2 ? TT_NP : kind == 3 ? CRN_NP : 0; }

void ionic_defaults(int kind, double *params)
{
    static const double ms[MS_NP] = {0.3, 6.0, 120.0, 150.0, 0.13, -80.0, 100.0};
    static const double tt[TT_NP] = {14.838, 5.405, 0.073, 0.153,  0.392,  3.98e-5,
                                     2.9e-4, 5.92e-4, 0.1238, 0.0146, 2.724, 1000.0};
    if (kind == 1)
        for (int i = 0; i < MS_NP; ++i) params[i] = ms[i];
    if (kind == 2)
        for (int i = 0; i < TT_NP; ++i) params[i] = tt[i];
    static const double crn_p[CRN_NP] = {7.8,     0.09,     0.1652,     0.029411765, 0.12941176,
                                         0.12375, 6.744375e-4, 1.131e-3, 0.59933874,  1600.0,
                                         0.275,   0.005,    1.0};
    if (kind == 3)
        for (int i = 0; i < CRN_NP; ++i) params[i] = crn_p[i];
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
    else if (kind == 3)
        hipLaunchKernelGGL(k_ionic_init<MDX_KIND_CRN>, grid, block, 0, s, P, n, ld, V, Vprev, u, tile_real);
    else
        hipLaunchKernelGGL(k_ionic_init<MDX_KIND_NONE>, grid, block, 0, s, P, n, ld, V, Vprev, u, tile_real);
}

void launch_ionic_step(hipStream_t s, int kind, const double *params, int64_t n, int64_t ld,
                       double dt, double cm, const double *V, double *u, const double *istim,
                       double *out, int raw, const int32_t *tile_real, const int32_t *guard,
                       const StepTimes &times)
{
    if (n <= 0) return;
    IonicParams P = pack(kind, params);
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (kind == 1)
        hipLaunchKernelGGL(k_ionic_step<MDX_KIND_MS>, grid, block, 0, s, P, n, ld, dt, cm, V, u,
                           istim, out, raw, tile_real, guard, times);
    else if (kind == 2)
        hipLaunchKernelGGL(k_ionic_step<MDX_KIND_TT>, grid, block, 0, s, P, n, ld, dt, cm, V, u,
                           istim, out, raw, tile_real, guard, times);
    else if (kind == 3)
        hipLaunchKernelGGL(k_ionic_step<MDX_KIND_CRN>, grid, block, 0, s, P, n, ld, dt, cm, V, u,
                           istim, out, raw, tile_real, guard, times);
    else
        hipLaunchKernelGGL(k_ionic_step<MDX_KIND_NONE>, grid, block, 0, s, P, n, ld, dt, cm, V, u,
                           istim, out, raw, tile_real, guard, times);
}

int ionic_gate_rows(int kind) { return kind == 1 ? 1 : kind == 2 ? 12 : 0; }
int ionic_gate_row0(int kind) { return kind == 1 ? 0 : kind == 2 ? 6 : 0; }

void launch_ionic_step_mixed(hipStream_t s, int kind, const double *params, int64_t n, int64_t ld,
                             double dt, double cm, const double *V, double *u, float *g32,
                             const double *istim, double *out, const int32_t *tile_real,
                             const int32_t *guard, const StepTimes &times)
{
    if (n <= 0) return;
    IonicParams P = pack(kind, params);
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (kind == 1)
        hipLaunchKernelGGL(k_ionic_step_mixed<MDX_KIND_MS>, grid, block, 0, s, P, n, ld, dt, cm, V,
                           u, g32, istim, out, tile_real, guard, times);
    else if (kind == 2)
        hipLaunchKernelGGL(k_ionic_step_mixed<MDX_KIND_TT>, grid, block, 0, s, P, n, ld, dt, cm, V,
                           u, g32, istim, out, tile_real, guard, times);
    else
        hipLaunchKernelGGL(k_ionic_step_mixed<MDX_KIND_NONE>, grid, block, 0, s, P, n, ld, dt, cm,
                           V, u, g32, istim, out, tile_real, guard, times);
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
