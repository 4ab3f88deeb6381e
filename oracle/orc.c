/*
 * CPU ORACLE for the monodomain finite-element hot path.  TEST INFRASTRUCTURE:
 * only the tests, the smoke check and the benchmark's CPU-baseline leg load
 * this file's library.  It shares no code with the HIP library.
 *
 * Plain, slow, FP64 C written from the paper (TorchCor, arXiv 2510.12011):
 *   - monodomain system and its theta-method discretisation: Eq. (1), Eq. (2)
 *     and the definitions of A and b that follow Eq. (3);
 *   - Jacobi-preconditioned CG: Algorithm 1, with the warm start
 *     x0 = 2V^k - V^{k-1} given after it;
 *   - activation / repolarisation times: "Software functionality" section;
 *   - P1 elements, transversely isotropic conductivity from longitudinal and
 *     transverse values along the element fibre: "Software functionality"
 *     and "Software implementation" sections.
 * The paper names its cell models but prints none of their equations; the two
 * used here are written from their original publications:
 *   - two-variable Mitchell-Schaeffer (Bull. Math. Biol. 65, 2003), gate by
 *     Rush-Larsen;
 *   - ten Tusscher-Panfilov 2006 endocardial (Am. J. Physiol. 291, H1088),
 *     12 gates by Rush-Larsen, 6 concentration-type states by forward Euler.
 * Readings where the paper is silent or inconsistent are stated at the point
 * of use (sign of the (1-theta) K term, order of the stopping test, ...).
 *
 * Parity status: assembly, PCG and time stepping are pinned by closed forms
 * and invariants in the CPU test suite; the ten Tusscher-Panfilov transcription
 * is "parity unpinned" against the literature (no published trace is available
 * offline) and is checked only qualitatively.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Sparsity pattern: row i holds every node sharing an element with i       */
/* (npe vertex ids per element: 4 for tetrahedra, 3 for surface triangles). */
/* Columns sorted ascending.  Returns nnz; fills col only if cap >= nnz.     */
/* ------------------------------------------------------------------------ */
static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

int64_t orc_pattern_elems(int64_t n, int64_t m, int npe, const int32_t *el,
                          int64_t *row_ptr, int32_t *col, int64_t cap)
{
    int64_t *cnt = calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t e = 0; e < m; ++e)
        for (int a = 0; a < npe; ++a) cnt[el[npe * e + a] + 1] += 1;
    for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)n);
    int32_t *inc = malloc(sizeof(int32_t) * (size_t)(cnt[n] > 0 ? cnt[n] : 1));
    memcpy(fill, cnt, sizeof(int64_t) * (size_t)n);
    for (int64_t e = 0; e < m; ++e)
        for (int a = 0; a < npe; ++a) inc[fill[el[npe * e + a]]++] = (int32_t)e;

    /* room for every vertex id of the most-shared node's elements */
    int64_t max_inc = 1;
    for (int64_t i = 0; i < n; ++i)
        if (cnt[i + 1] - cnt[i] > max_inc) max_inc = cnt[i + 1] - cnt[i];
    int32_t *buf = malloc(sizeof(int32_t) * (size_t)(npe * max_inc));
    int64_t nnz = 0;
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t nb = 0;
        for (int64_t t = cnt[i]; t < cnt[i + 1]; ++t)
            for (int a = 0; a < npe; ++a) buf[nb++] = el[npe * (int64_t)inc[t] + a];
        if (nb == 0) buf[nb++] = (int32_t)i; /* isolated node keeps its diagonal */
        qsort(buf, (size_t)nb, sizeof(int32_t), cmp_i32);
        int64_t nu = 0;
        for (int64_t q = 0; q < nb; ++q)
            if (q == 0 || buf[q] != buf[q - 1]) buf[nu++] = buf[q];
        if (col && nnz + nu <= cap) memcpy(col + nnz, buf, sizeof(int32_t) * (size_t)nu);
        nnz += nu;
        row_ptr[i + 1] = nnz;
    }
    free(cnt); free(fill); free(inc); free(buf);
    return nnz;
}

int64_t orc_pattern(int64_t n, int64_t m, const int32_t *tets,
                    int64_t *row_ptr, int32_t *col, int64_t cap)
{
    return orc_pattern_elems(n, m, 4, tets, row_ptr, col, cap);
}

/* ------------------------------------------------------------------------ */
/* Element matrices of a P1 tetrahedron.                                     */
/*   J = [x1-x0, x2-x0, x3-x0] (columns), vol = |det J| / 6;                 */
/*   grad phi_{c+1} = row c of J^{-1}, grad phi_0 = -sum of the others;     */
/*   sigma = st I + (sl - st) f f^T with f the unit fibre (isotropic st if   */
/*   no fibre); K_e[a][b] = vol * grad phi_a . sigma grad phi_b;             */
/*   M_e[a][b] = vol/20 * (1 + delta_ab)  (exact consistent P1 mass).        */
/* Returns the signed determinant of J.                                      */
/* ------------------------------------------------------------------------ */
double orc_element(const double *p0, const double *p1, const double *p2,
                   const double *p3, const double *fib, double sl, double st,
                   double *Me, double *Ke)
{
    double J[3][3];
    for (int r = 0; r < 3; ++r) {
        J[r][0] = p1[r] - p0[r];
        J[r][1] = p2[r] - p0[r];
        J[r][2] = p3[r] - p0[r];
    }
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
               - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
               + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    /* inverse via the adjugate: Jinv[i][j] = cofactor(j,i) / det */
    double Ji[3][3];
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    double vol = fabs(det) / 6.0;

    double g[4][3];
    for (int c = 0; c < 3; ++c) {
        g[c + 1][0] = Ji[c][0];
        g[c + 1][1] = Ji[c][1];
        g[c + 1][2] = Ji[c][2];
    }
    for (int d = 0; d < 3; ++d) g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);

    double f[3] = {0.0, 0.0, 0.0};
    double fn = 0.0;
    if (fib) fn = sqrt(fib[0] * fib[0] + fib[1] * fib[1] + fib[2] * fib[2]);
    if (fn > 0.0) { f[0] = fib[0] / fn; f[1] = fib[1] / fn; f[2] = fib[2] / fn; }
    double S[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            S[r][c] = (r == c ? st : 0.0) + (sl - st) * f[r] * f[c];

    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            double s = 0.0;
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) s += g[a][r] * S[r][c] * g[b][c];
            Ke[4 * a + b] = vol * s;
            Me[4 * a + b] = vol / 20.0 * (a == b ? 2.0 : 1.0);
        }
    return det;
}

static int64_t find_slot(const int64_t *row_ptr, const int32_t *col, int64_t i, int32_t j)
{
    int64_t lo = row_ptr[i], hi = row_ptr[i + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (col[mid] == j) return mid;
        if (col[mid] < j) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* Global M and K on the pattern from orc_pattern; sl/st are per element.
 * Returns 0, or -(e+1) for the first element e with non-positive volume. */
int64_t orc_assemble(int64_t n, const double *xyz, int64_t m, const int32_t *tets,
                     const double *fibre, const double *sl, const double *st,
                     const int64_t *row_ptr, const int32_t *col,
                     double *Mv, double *Kv)
{
    memset(Mv, 0, sizeof(double) * (size_t)row_ptr[n]);
    memset(Kv, 0, sizeof(double) * (size_t)row_ptr[n]);
    double Me[16], Ke[16];
    for (int64_t e = 0; e < m; ++e) {
        const int32_t *t = tets + 4 * e;
        double det = orc_element(xyz + 3 * t[0], xyz + 3 * t[1], xyz + 3 * t[2],
                                 xyz + 3 * t[3], fibre ? fibre + 3 * e : NULL,
                                 sl[e], st[e], Me, Ke);
        if (!(fabs(det) > 0.0)) return -(e + 1);
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                int64_t s = find_slot(row_ptr, col, t[a], t[b]);
                Mv[s] += Me[4 * a + b];
                Kv[s] += Ke[4 * a + b];
            }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Element matrices of a P1 triangle of a surface mesh in 3D (the paper's    */
/* "Software functionality" section admits triangular as well as           */
/* tetrahedral elements).  With the edge matrix E = [x1-x0, x2-x0] (3x2)     */
/* and its metric G = E^T E:                                                 */
/*   area = sqrt(det G) / 2;                                                 */
/*   the surface gradient of phi_a is E G^{-1} d_a, with the reference      */
/*   gradients d_0 = (-1,-1), d_1 = (1,0), d_2 = (0,1);                      */
/*   sigma = st I + (sl - st) f f^T, f the fibre's projection on the         */
/*   triangle's plane, E G^{-1} E^T fib, normalised (isotropic st if there   */
/*   is no fibre or it is normal to the triangle);                           */
/*   K_e[a][b] = area * grad phi_a . sigma grad phi_b;                       */
/*   M_e[a][b] = area/12 * (1 + delta_ab)  (exact consistent P1 mass).       */
/* Me, Ke: 3x3 row-major.  Returns det G (zero for a degenerate triangle).   */
/* ------------------------------------------------------------------------ */
double orc_element_tri(const double *p0, const double *p1, const double *p2,
                       const double *fib, double sl, double st, double *Me, double *Ke)
{
    double E[3][2];
    for (int r = 0; r < 3; ++r) {
        E[r][0] = p1[r] - p0[r];
        E[r][1] = p2[r] - p0[r];
    }
    double G[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int r = 0; r < 3; ++r) G[i][j] += E[r][i] * E[r][j];
    double detG = G[0][0] * G[1][1] - G[0][1] * G[1][0];
    if (!(detG > 0.0)) return 0.0;
    double Gi[2][2] = {{G[1][1] / detG, -G[0][1] / detG}, {-G[1][0] / detG, G[0][0] / detG}};
    double area = 0.5 * sqrt(detG);
    /* E G^{-1} (3x2): maps reference gradients to surface gradients */
    double EGi[3][2];
    for (int r = 0; r < 3; ++r)
        for (int j = 0; j < 2; ++j) EGi[r][j] = E[r][0] * Gi[0][j] + E[r][1] * Gi[1][j];
    const double d[3][2] = {{-1.0, -1.0}, {1.0, 0.0}, {0.0, 1.0}};
    double g[3][3];
    for (int a = 0; a < 3; ++a)
        for (int r = 0; r < 3; ++r) g[a][r] = EGi[r][0] * d[a][0] + EGi[r][1] * d[a][1];

    double f[3] = {0.0, 0.0, 0.0};
    if (fib) {
        double Etf[2] = {0.0, 0.0};
        for (int j = 0; j < 2; ++j)
            for (int r = 0; r < 3; ++r) Etf[j] += E[r][j] * fib[r];
        double pf[3], pn = 0.0;
        for (int r = 0; r < 3; ++r) {
            pf[r] = EGi[r][0] * Etf[0] + EGi[r][1] * Etf[1];
            pn += pf[r] * pf[r];
        }
        pn = sqrt(pn);
        double fn = sqrt(fib[0] * fib[0] + fib[1] * fib[1] + fib[2] * fib[2]);
        /* a fibre (numerically) normal to the triangle leaves it isotropic */
        if (pn > 1e-12 * fn)
            for (int r = 0; r < 3; ++r) f[r] = pf[r] / pn;
    }
    double S[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            S[r][c] = (r == c ? st : 0.0) + (sl - st) * f[r] * f[c];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) s += g[a][r] * S[r][c] * g[b][c];
            Ke[3 * a + b] = area * s;
            Me[3 * a + b] = area / 12.0 * (a == b ? 2.0 : 1.0);
        }
    return detG;
}

/* Global M and K of a triangle surface mesh on the pattern from
 * orc_pattern_elems (npe = 3).  Returns 0, or -(e+1) for the first
 * degenerate triangle e. */
int64_t orc_assemble_tri(int64_t n, const double *xyz, int64_t m, const int32_t *tris,
                         const double *fibre, const double *sl, const double *st,
                         const int64_t *row_ptr, const int32_t *col,
                         double *Mv, double *Kv)
{
    memset(Mv, 0, sizeof(double) * (size_t)row_ptr[n]);
    memset(Kv, 0, sizeof(double) * (size_t)row_ptr[n]);
    double Me[9], Ke[9];
    for (int64_t e = 0; e < m; ++e) {
        const int32_t *t = tris + 3 * e;
        double detG = orc_element_tri(xyz + 3 * t[0], xyz + 3 * t[1], xyz + 3 * t[2],
                                      fibre ? fibre + 3 * e : NULL, sl[e], st[e], Me, Ke);
        if (!(detG > 0.0)) return -(e + 1);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                int64_t s = find_slot(row_ptr, col, t[a], t[b]);
                Mv[s] += Me[3 * a + b];
                Kv[s] += Ke[3 * a + b];
            }
    }
    return 0;
}

/* y = A x for CSR A */
void orc_spmv(int64_t n, const int64_t *row_ptr, const int32_t *col,
              const double *val, const double *x, double *y)
{
#pragma omp parallel for schedule(static) if (n > 20000)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) s += val[q] * x[col[q]];
        y[i] = s;
    }
}

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* ------------------------------------------------------------------------ */
/* Jacobi-PCG, Algorithm 1.  Readings of the printed algorithm:              */
/*  - z_{k+1} = D^{-1} r_{k+1} is formed before the stopping test that uses  */
/*    its norm (the printed order tests it one line before forming it);      */
/*  - the relative test compares ||z_{k+1}|| with the initial ||z_0||        */
/*    (rel_mode 0, the paper's) or with ||D^{-1} b|| (rel_mode 1);           */
/*  - a floor ||z|| <= 1e-15 ||D^{-1} b|| also stops (a rounding-level       */
/*    residual cannot shrink further), also before the first iteration.      */
/* x holds x0 on entry and the solution on exit.  Returns the iteration      */
/* count, or -1 if max_iter was reached without meeting the test.            */
/* ------------------------------------------------------------------------ */
int orc_pcg(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *A,
            const double *b, double *x, double atol, double rtol, int rel_mode,
            int max_iter, double *final_znorm)
{
    double *dinv = malloc(sizeof(double) * (size_t)n);
    double *r = malloc(sizeof(double) * (size_t)n);
    double *z = malloc(sizeof(double) * (size_t)n);
    double *p = malloc(sizeof(double) * (size_t)n);
    double *q = malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int64_t s = row_ptr[i]; s < row_ptr[i + 1]; ++s)
            if (col[s] == i) d = A[s];
        dinv[i] = 1.0 / d;
    }
    orc_spmv(n, row_ptr, col, A, x, q);
    for (int64_t i = 0; i < n; ++i) {
        r[i] = b[i] - q[i];
        z[i] = dinv[i] * r[i];
        p[i] = z[i];
        q[i] = dinv[i] * b[i];           /* q used as scratch for D^-1 b */
    }
    double rho = dot(n, r, z);
    double z0 = sqrt(dot(n, z, z));
    double db = sqrt(dot(n, q, q));
    double ref = rel_mode == 0 ? z0 : db;
    double floor_ = 1e-15 * db;
    int it = 0, conv = 0;
    double zn = z0;
    if (z0 <= floor_ || z0 < atol) conv = 1;
    while (!conv && it < max_iter) {
        orc_spmv(n, row_ptr, col, A, p, q);
        double alpha = rho / dot(n, p, q);
        for (int64_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
            z[i] = dinv[i] * r[i];
        }
        ++it;
        zn = sqrt(dot(n, z, z));
        if (zn < atol || zn < rtol * ref || zn <= floor_) { conv = 1; break; }
        double rho1 = dot(n, r, z);
        double beta = rho1 / rho;
        rho = rho1;
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    if (final_znorm) *final_znorm = zn;
    free(dinv); free(r); free(z); free(p); free(q);
    return conv ? it : -1;
}

/* ------------------------------------------------------------------------ */
/* Mitchell-Schaeffer two-variable model in the monodomain's units.          */
/* params: tau_in, tau_out, tau_open, tau_close, u_gate, v_rest, v_amp.      */
/* u = (V - v_rest)/v_amp;  dh/dt = (1-h)/tau_open if u < u_gate, else      */
/* -h/tau_close (advanced by Rush-Larsen, which is exact for frozen u);      */
/* current per unit capacitance (mV/ms):                                     */
/*   Iion/Cm = -v_amp * ( h u^2 (1-u) / tau_in - u / tau_out ).              */
/* ------------------------------------------------------------------------ */
#define MS_NPAR 7
static const double MS_DEFAULT[MS_NPAR] = {0.3, 6.0, 120.0, 150.0, 0.13, -80.0, 100.0};

static void ms_point(const double *pr, double dt, double V, double *h, double *iion)
{
    double u = (V - pr[5]) / pr[6];
    double hinf, tau;
    if (u < pr[4]) { hinf = 1.0; tau = pr[2]; } else { hinf = 0.0; tau = pr[3]; }
    *h = hinf + (*h - hinf) * exp(-dt / tau);
    *iion = -pr[6] * (*h * u * u * (1.0 - u) / pr[0] - u / pr[1]);
}

/* ------------------------------------------------------------------------ */
/* ten Tusscher-Panfilov 2006, endocardial cell.  States (index):            */
/*  0 Ki 1 Nai 2 Cai 3 CaSR 4 CaSS 5 Rbar 6 xr1 7 xr2 8 xs 9 m 10 h 11 j     */
/*  12 d 13 f 14 f2 15 fCass 16 s 17 r.  V in mV, t in ms, currents pA/pF.   */
/* params (scale the maximal conductances / fluxes; defaults below):         */
/*  0 GNa 1 GK1 2 Gto 3 GKr 4 GKs 5 GCaL 6 GbNa 7 GbCa 8 GpCa 9 GpK          */
/*  10 PNaK 11 kNaCa                                                         */
/* ------------------------------------------------------------------------ */
#define TT_NS 18
#define TT_NPAR 12
static const double TT_DEFAULT[TT_NPAR] = {14.838, 5.405, 0.073, 0.153, 0.392, 3.98e-5,
                                           2.9e-4, 5.92e-4, 0.1238, 0.0146, 2.724, 1000.0};
static const double TT_INIT[TT_NS] = {136.89, 8.604, 0.000126, 3.64, 0.00036, 0.9073,
                                      0.00621, 0.4712, 0.0095, 0.00172, 0.7444, 0.7045,
                                      3.373e-5, 0.7888, 0.9755, 0.9953, 0.999998, 2.42e-8};
static const double TT_V0 = -85.23;

/* physical constants and fixed model constants */
#define TT_R 8314.472
#define TT_T 310.0
#define TT_F 96485.3415
#define TT_CAP 0.185
#define TT_VC 0.016404
#define TT_VSR 0.001094
#define TT_VSS 0.00005468
#define TT_KO 5.4
#define TT_NAO 140.0
#define TT_CAO 2.0
#define TT_PKNA 0.03
#define TT_KMK 1.0
#define TT_KMNA 40.0
#define TT_KMNAI 87.5
#define TT_KMCA 1.38
#define TT_KSAT 0.1
#define TT_GAMMA 0.35
#define TT_ALPHA 2.5
#define TT_KPCA 0.0005
#define TT_BUFC 0.2
#define TT_KBUFC 0.001
#define TT_BUFSR 10.0
#define TT_KBUFSR 0.3
#define TT_BUFSS 0.4
#define TT_KBUFSS 0.00025
#define TT_VMAXUP 0.006375
#define TT_KUP 0.00025
#define TT_VREL 0.102
#define TT_K1P 0.15
#define TT_K2P 0.045
#define TT_K3 0.06
#define TT_K4 0.005
#define TT_EC 1.5
#define TT_MAXSR 2.5
#define TT_MINSR 1.0
#define TT_VLEAK 0.00036
#define TT_VXFER 0.0038

typedef struct {
    double IK1, Ito, IKr, IKs, ICaL, INaK, INa, IbNa, INaCa, IbCa, IpK, IpCa;
} tt_currents;

static void tt_currents_at(const double *g, double V, const double *y, tt_currents *c)
{
    const double RTF = TT_R * TT_T / TT_F;
    double Ki = y[0], Nai = y[1], Cai = y[2], CaSS = y[4];
    double EK = RTF * log(TT_KO / Ki);
    double ENa = RTF * log(TT_NAO / Nai);
    double EKs = RTF * log((TT_KO + TT_PKNA * TT_NAO) / (Ki + TT_PKNA * Nai));
    double ECa = 0.5 * RTF * log(TT_CAO / Cai);

    double aK1 = 0.1 / (1.0 + exp(0.06 * (V - EK - 200.0)));
    double bK1 = (3.0 * exp(0.0002 * (V - EK + 100.0)) + exp(0.1 * (V - EK - 10.0)))
               / (1.0 + exp(-0.5 * (V - EK)));
    double xK1 = aK1 / (aK1 + bK1);
    double sk = sqrt(TT_KO / 5.4);
    c->IK1 = g[1] * sk * xK1 * (V - EK);
    c->Ito = g[2] * y[17] * y[16] * (V - EK);
    c->IKr = g[3] * sk * y[6] * y[7] * (V - EK);
    c->IKs = g[4] * y[8] * y[8] * (V - EKs);
    c->INa = g[0] * y[9] * y[9] * y[9] * y[10] * y[11] * (V - ENa);
    c->IbNa = g[6] * (V - ENa);
    c->IbCa = g[7] * (V - ECa);
    /* L-type: 4 (V-15) F^2/(RT) (0.25 CaSS e^w - Cao)/(e^w - 1), w = 2(V-15)F/RT;
     * (V-15)/(e^w - 1) is written as (RT/2F) w/expm1(w), limit 1 at w = 0 */
    double w = 2.0 * (V - 15.0) / RTF;
    double wq = (w == 0.0) ? 1.0 : w / expm1(w);
    c->ICaL = g[5] * y[12] * y[13] * y[14] * y[15] * 2.0 * TT_F * wq
            * (0.25 * CaSS * exp(w) - TT_CAO);
    double vf = V / RTF;
    c->INaK = g[10] * TT_KO / (TT_KO + TT_KMK) * Nai / (Nai + TT_KMNA)
            / (1.0 + 0.1245 * exp(-0.1 * vf) + 0.0353 * exp(-vf));
    c->INaCa = g[11] * (exp(TT_GAMMA * vf) * Nai * Nai * Nai * TT_CAO
                        - exp((TT_GAMMA - 1.0) * vf) * TT_NAO * TT_NAO * TT_NAO * Cai * TT_ALPHA)
             / ((TT_KMNAI * TT_KMNAI * TT_KMNAI + TT_NAO * TT_NAO * TT_NAO) * (TT_KMCA + TT_CAO)
                * (1.0 + TT_KSAT * exp((TT_GAMMA - 1.0) * vf)));
    c->IpCa = g[8] * Cai / (TT_KPCA + Cai);
    c->IpK = g[9] * (V - EK) / (1.0 + exp((25.0 - V) / 5.98));
}

static double tt_sum(const tt_currents *c)
{
    return c->IK1 + c->Ito + c->IKr + c->IKs + c->ICaL + c->INaK + c->INa + c->IbNa
         + c->INaCa + c->IbCa + c->IpK + c->IpCa;
}

static double rl(double y, double yinf, double tau, double dt)
{
    return yinf - (yinf - y) * exp(-dt / tau);
}

static void tt_point(const double *g, double dt, double V, double *y, double *iion)
{
    tt_currents c;
    tt_currents_at(g, V, y, &c);
    double Cai = y[2], CaSR = y[3], CaSS = y[4], Rb = y[5];

    /* calcium handling, derivatives at (V^k, u^k) */
    double kcasr = TT_MAXSR - (TT_MAXSR - TT_MINSR) / (1.0 + (TT_EC / CaSR) * (TT_EC / CaSR));
    double k1 = TT_K1P / kcasr, k2 = TT_K2P * kcasr;
    double O = k1 * CaSS * CaSS * Rb / (TT_K3 + k1 * CaSS * CaSS);
    double dRb = -k2 * CaSS * Rb + TT_K4 * (1.0 - Rb);
    double Irel = TT_VREL * O * (CaSR - CaSS);
    double Iup = TT_VMAXUP / (1.0 + TT_KUP * TT_KUP / (Cai * Cai));
    double Ileak = TT_VLEAK * (CaSR - Cai);
    double Ixfer = TT_VXFER * (CaSS - Cai);
    double bc = 1.0 / (1.0 + TT_BUFC * TT_KBUFC / ((Cai + TT_KBUFC) * (Cai + TT_KBUFC)));
    double bsr = 1.0 / (1.0 + TT_BUFSR * TT_KBUFSR / ((CaSR + TT_KBUFSR) * (CaSR + TT_KBUFSR)));
    double bss = 1.0 / (1.0 + TT_BUFSS * TT_KBUFSS / ((CaSS + TT_KBUFSS) * (CaSS + TT_KBUFSS)));
    double dCai = bc * ((Ileak - Iup) * TT_VSR / TT_VC + Ixfer
                        - (c.IbCa + c.IpCa - 2.0 * c.INaCa) * TT_CAP / (2.0 * TT_VC * TT_F));
    double dCaSR = bsr * (Iup - Irel - Ileak);
    double dCaSS = bss * (-c.ICaL * TT_CAP / (2.0 * TT_VSS * TT_F) + Irel * TT_VSR / TT_VSS
                          - Ixfer * TT_VC / TT_VSS);
    double dNai = -(c.INa + c.IbNa + 3.0 * c.INaK + 3.0 * c.INaCa) * TT_CAP / (TT_VC * TT_F);
    double dKi = -(c.IK1 + c.Ito + c.IKr + c.IKs - 2.0 * c.INaK + c.IpK) * TT_CAP / (TT_VC * TT_F);

    /* gates: steady state and time constant at V^k */
    double minf = 1.0 / ((1.0 + exp((-56.86 - V) / 9.03)) * (1.0 + exp((-56.86 - V) / 9.03)));
    double am = 1.0 / (1.0 + exp((-60.0 - V) / 5.0));
    double bm = 0.1 / (1.0 + exp((V + 35.0) / 5.0)) + 0.1 / (1.0 + exp((V - 50.0) / 200.0));
    double tm = am * bm;
    double hinf = 1.0 / ((1.0 + exp((V + 71.55) / 7.43)) * (1.0 + exp((V + 71.55) / 7.43)));
    double ah, bh, aj, bj;
    if (V >= -40.0) {
        ah = 0.0;
        bh = 0.77 / (0.13 * (1.0 + exp(-(V + 10.66) / 11.1)));
        aj = 0.0;
        bj = 0.6 * exp(0.057 * V) / (1.0 + exp(-0.1 * (V + 32.0)));
    } else {
        ah = 0.057 * exp(-(V + 80.0) / 6.8);
        bh = 2.7 * exp(0.079 * V) + 3.1e5 * exp(0.3485 * V);
        aj = (-25428.0 * exp(0.2444 * V) - 6.948e-6 * exp(-0.04391 * V)) * (V + 37.78)
           / (1.0 + exp(0.311 * (V + 79.23)));
        bj = 0.02424 * exp(-0.01052 * V) / (1.0 + exp(-0.1378 * (V + 40.14)));
    }
    double th = 1.0 / (ah + bh), tj = 1.0 / (aj + bj);
    double xr1inf = 1.0 / (1.0 + exp((-26.0 - V) / 7.0));
    double txr1 = (450.0 / (1.0 + exp((-45.0 - V) / 10.0))) * (6.0 / (1.0 + exp((V + 30.0) / 11.5)));
    double xr2inf = 1.0 / (1.0 + exp((V + 88.0) / 24.0));
    double txr2 = (3.0 / (1.0 + exp((-60.0 - V) / 20.0))) * (1.12 / (1.0 + exp((V - 60.0) / 20.0)));
    double xsinf = 1.0 / (1.0 + exp((-5.0 - V) / 14.0));
    double txs = (1400.0 / sqrt(1.0 + exp((5.0 - V) / 6.0))) * (1.0 / (1.0 + exp((V - 35.0) / 15.0))) + 80.0;
    double rinf = 1.0 / (1.0 + exp((20.0 - V) / 6.0));
    double tr = 9.5 * exp(-(V + 40.0) * (V + 40.0) / 1800.0) + 0.8;
    double sinf = 1.0 / (1.0 + exp((V + 28.0) / 5.0));
    double ts = 1000.0 * exp(-(V + 67.0) * (V + 67.0) / 1000.0) + 8.0;
    double dinf = 1.0 / (1.0 + exp((-8.0 - V) / 7.5));
    double ad = 1.4 / (1.0 + exp((-35.0 - V) / 13.0)) + 0.25;
    double bd = 1.4 / (1.0 + exp((V + 5.0) / 5.0));
    double gd = 1.0 / (1.0 + exp((50.0 - V) / 20.0));
    double td = ad * bd + gd;
    double finf = 1.0 / (1.0 + exp((V + 20.0) / 7.0));
    double tf = 1102.5 * exp(-(V + 27.0) * (V + 27.0) / 225.0) + 200.0 / (1.0 + exp((13.0 - V) / 10.0))
              + 180.0 / (1.0 + exp((V + 30.0) / 10.0)) + 20.0;
    double f2inf = 0.67 / (1.0 + exp((V + 35.0) / 7.0)) + 0.33;
    double tf2 = 562.0 * exp(-(V + 27.0) * (V + 27.0) / 240.0) + 31.0 / (1.0 + exp((25.0 - V) / 10.0))
               + 80.0 / (1.0 + exp((V + 30.0) / 10.0));
    double cs = (CaSS / 0.05) * (CaSS / 0.05);
    double fcinf = 0.6 / (1.0 + cs) + 0.4;
    double tfc = 80.0 / (1.0 + cs) + 2.0;

    /* forward Euler for the concentration-type states */
    y[0] += dt * dKi;
    y[1] += dt * dNai;
    y[2] += dt * dCai;
    y[3] += dt * dCaSR;
    y[4] += dt * dCaSS;
    y[5] += dt * dRb;
    /* Rush-Larsen for the gates */
    y[6] = rl(y[6], xr1inf, txr1, dt);
    y[7] = rl(y[7], xr2inf, txr2, dt);
    y[8] = rl(y[8], xsinf, txs, dt);
    y[9] = rl(y[9], minf, tm, dt);
    y[10] = rl(y[10], hinf, th, dt);
    y[11] = rl(y[11], hinf, tj, dt);
    y[12] = rl(y[12], dinf, td, dt);
    y[13] = rl(y[13], finf, tf, dt);
    y[14] = rl(y[14], f2inf, tf2, dt);
    y[15] = rl(y[15], fcinf, tfc, dt);
    y[16] = rl(y[16], sinf, ts, dt);
    y[17] = rl(y[17], rinf, tr, dt);

    /* I_ion(V^k, u^{k+1}) */
    tt_currents_at(g, V, y, &c);
    *iion = tt_sum(&c);
}

/* ------------------------------------------------------------------------ */
/* Courtemanche-Ramirez-Nattel 1998 human atrial cell (the atrial model the  */
/* paper's "Software implementation" section names), from the published     */
/* equations.  States (index):                                               */
/*  0 Nai 1 Ki 2 Cai 3 Caup 4 Carel 5 m 6 h 7 j 8 oa 9 oi 10 ua 11 ui        */
/*  12 xr 13 xs 14 d 15 f 16 fCa 17 u 18 v 19 w.  V in mV, t in ms; currents */
/*  per unit capacitance (pA/pF = mV/ms), concentrations mM, volumes um^3.   */
/* params: 0 gNa 1 gK1 2 gto 3 gKr 4 gKs 5 gCaL 6 gbNa 7 gbCa (nS/pF)        */
/*  8 INaK_max 9 INaCa_max 10 IpCa_max (pA/pF) 11 Iup_max (mM/ms)            */
/*  12 scale of the ultrarapid K conductance gKur(V)                         */
/* ------------------------------------------------------------------------ */
#define CRN_NS 20
#define CRN_NPAR 13
static const double CRN_DEFAULT[CRN_NPAR] = {7.8, 0.09, 0.1652, 0.029411765, 0.12941176,
                                             0.12375, 6.744375e-4, 1.131e-3, 0.59933874,
                                             1600.0, 0.275, 0.005, 1.0};
static const double CRN_INIT[CRN_NS] = {11.17, 139.0, 1.013e-4, 1.488, 1.488,
                                        2.908e-3, 0.9649, 0.9775, 3.043e-2, 0.9992,
                                        4.966e-3, 0.9986, 3.296e-5, 1.869e-2, 1.367e-4,
                                        0.9996, 0.7755, 0.0, 1.0, 0.9992};
static const double CRN_V0 = -81.18;
#define CRN_R 8.3143
#define CRN_T 310.0
#define CRN_F 96.4867
#define CRN_CM 100.0          /* pF */
#define CRN_VI 13668.0
#define CRN_VUP 1109.52
#define CRN_VREL 96.48
#define CRN_KO 5.4
#define CRN_NAO 140.0
#define CRN_CAO 1.8
#define CRN_KMNAI 10.0        /* I_NaK half-saturation in Na_i */
#define CRN_KMKO 1.5          /* I_NaK half-saturation in K_o */
#define CRN_KMNA 87.5         /* I_NaCa */
#define CRN_KMCA 1.38
#define CRN_KSAT 0.1
#define CRN_GAMMA 0.35
#define CRN_KREL 30.0
#define CRN_KUP 0.00092
#define CRN_CAUPMAX 15.0
#define CRN_TAUTR 180.0
#define CRN_CMDN 0.05
#define CRN_TRPN 0.07
#define CRN_CSQN 10.0
#define CRN_KMCMDN 0.00238
#define CRN_KMTRPN 0.0005
#define CRN_KMCSQN 0.8
#define CRN_KQ10 3.0

/* x / (1 - exp(-x/s)) and x / (exp(x/s) - 1), with their limits s at x = 0 */
static double crn_x_over_1mexp(double x, double s)
{
    double t = x / s;
    return t == 0.0 ? s : -x / expm1(-t);
}
static double crn_x_over_expm1(double x, double s)
{
    double t = x / s;
    return t == 0.0 ? s : x / expm1(t);
}

typedef struct {
    double INa, IK1, Ito, IKur, IKr, IKs, ICaL, INaK, INaCa, IbNa, IbCa, IpCa;
} crn_currents;

static void crn_currents_at(const double *g, double V, const double *y, crn_currents *c)
{
    const double RTF = CRN_R * CRN_T / CRN_F;
    double Nai = y[0], Ki = y[1], Cai = y[2];
    double ENa = RTF * log(CRN_NAO / Nai);
    double EK = RTF * log(CRN_KO / Ki);
    double ECa = 0.5 * RTF * log(CRN_CAO / Cai);
    double vf = V / RTF;
    c->INa = g[0] * y[5] * y[5] * y[5] * y[6] * y[7] * (V - ENa);
    c->IK1 = g[1] * (V - EK) / (1.0 + exp(0.07 * (V + 80.0)));
    c->Ito = g[2] * y[8] * y[8] * y[8] * y[9] * (V - EK);
    double gKur = g[12] * (0.005 + 0.05 / (1.0 + exp(-(V - 15.0) / 13.0)));
    c->IKur = gKur * y[10] * y[10] * y[10] * y[11] * (V - EK);
    c->IKr = g[3] * y[12] * (V - EK) / (1.0 + exp((V + 15.0) / 22.4));
    c->IKs = g[4] * y[13] * y[13] * (V - EK);
    c->ICaL = g[5] * y[14] * y[15] * y[16] * (V - 65.0);
    double sigma = (exp(CRN_NAO / 67.3) - 1.0) / 7.0;
    double fNaK = 1.0 / (1.0 + 0.1245 * exp(-0.1 * vf) + 0.0365 * sigma * exp(-vf));
    c->INaK = g[8] * fNaK / (1.0 + pow(CRN_KMNAI / Nai, 1.5)) * CRN_KO / (CRN_KO + CRN_KMKO);
    c->INaCa = g[9] * (exp(CRN_GAMMA * vf) * Nai * Nai * Nai * CRN_CAO
                       - exp((CRN_GAMMA - 1.0) * vf) * CRN_NAO * CRN_NAO * CRN_NAO * Cai)
             / ((CRN_KMNA * CRN_KMNA * CRN_KMNA + CRN_NAO * CRN_NAO * CRN_NAO)
                * (CRN_KMCA + CRN_CAO) * (1.0 + CRN_KSAT * exp((CRN_GAMMA - 1.0) * vf)));
    c->IbNa = g[6] * (V - ENa);
    c->IbCa = g[7] * (V - ECa);
    c->IpCa = g[10] * Cai / (0.0005 + Cai);
}

static double crn_sum(const crn_currents *c)
{
    return c->INa + c->IK1 + c->Ito + c->IKur + c->IKr + c->IKs + c->ICaL + c->INaK
         + c->INaCa + c->IbNa + c->IbCa + c->IpCa;
}

static void crn_point(const double *g, double dt, double V, double *y, double *iion)
{
    crn_currents c;
    crn_currents_at(g, V, y, &c);
    double Nai = y[0], Cai = y[2], Caup = y[3], Carel = y[4];
    (void)Nai;
    /* SR fluxes (mM/ms) and concentrations, derivatives at (V^k, u^k);
     * currents in pA are the per-capacitance values times Cm */
    double Irel = CRN_KREL * y[17] * y[17] * y[18] * y[19] * (Carel - Cai);
    double Itr = (Caup - Carel) / CRN_TAUTR;
    double Iup = g[11] / (1.0 + CRN_KUP / Cai);
    double Iupleak = g[11] * Caup / CRN_CAUPMAX;
    double FV = CRN_F * CRN_VI;
    double dNai = -CRN_CM * (3.0 * c.INaK + 3.0 * c.INaCa + c.IbNa + c.INa) / FV;
    double dKi = CRN_CM * (2.0 * c.INaK - (c.IK1 + c.Ito + c.IKur + c.IKr + c.IKs)) / FV;
    double B1 = CRN_CM * (2.0 * c.INaCa - (c.IpCa + c.ICaL + c.IbCa)) / (2.0 * FV)
              + (CRN_VUP * (Iupleak - Iup) + Irel * CRN_VREL) / CRN_VI;
    double B2 = 1.0 + CRN_TRPN * CRN_KMTRPN / ((Cai + CRN_KMTRPN) * (Cai + CRN_KMTRPN))
              + CRN_CMDN * CRN_KMCMDN / ((Cai + CRN_KMCMDN) * (Cai + CRN_KMCMDN));
    double dCai = B1 / B2;
    double dCaup = Iup - Iupleak - Itr * CRN_VREL / CRN_VUP;
    double dCarel = (Itr - Irel)
                  / (1.0 + CRN_CSQN * CRN_KMCSQN / ((Carel + CRN_KMCSQN) * (Carel + CRN_KMCSQN)));

    /* gates at V^k (and at Fn, Ca_i of step k for u, v, fCa) */
    double am = 0.32 * crn_x_over_1mexp(V + 47.13, 10.0);
    double bm = 0.08 * exp(-V / 11.0);
    double ah, bh, aj, bj;
    if (V < -40.0) {
        ah = 0.135 * exp((V + 80.0) / -6.8);
        bh = 3.56 * exp(0.079 * V) + 3.1e5 * exp(0.35 * V);
        aj = (-127140.0 * exp(0.2444 * V) - 3.474e-5 * exp(-0.04391 * V)) * (V + 37.78)
           / (1.0 + exp(0.311 * (V + 79.23)));
        bj = 0.1212 * exp(-0.01052 * V) / (1.0 + exp(-0.1378 * (V + 40.14)));
    } else {
        ah = 0.0;
        bh = 1.0 / (0.13 * (1.0 + exp((V + 10.66) / -11.1)));
        aj = 0.0;
        bj = 0.3 * exp(-2.535e-7 * V) / (1.0 + exp(-0.1 * (V + 32.0)));
    }
    double a_oa = 0.65 / (exp((V + 10.0) / -8.5) + exp((V - 30.0) / -59.0));
    double b_oa = 0.65 / (2.5 + exp((V + 82.0) / 17.0));
    double t_oa = 1.0 / ((a_oa + b_oa) * CRN_KQ10);
    double oainf = 1.0 / (1.0 + exp((V + 20.47) / -17.54));
    double a_oi = 1.0 / (18.53 + exp((V + 113.7) / 10.95));
    double b_oi = 1.0 / (35.56 + exp((V + 1.26) / -7.44));
    double t_oi = 1.0 / ((a_oi + b_oi) * CRN_KQ10);
    double oiinf = 1.0 / (1.0 + exp((V + 43.1) / 5.3));
    /* the ultrarapid activation gate has the transient one's rates */
    double t_ua = t_oa;
    double uainf = 1.0 / (1.0 + exp((V + 30.3) / -9.6));
    double a_ui = 1.0 / (21.0 + exp((V - 185.0) / -28.0));
    double b_ui = exp((V - 158.0) / 16.0);
    double t_ui = 1.0 / ((a_ui + b_ui) * CRN_KQ10);
    double uiinf = 1.0 / (1.0 + exp((V - 99.45) / 27.48));
    double a_xr = 0.0003 * crn_x_over_1mexp(V + 14.1, 5.0);
    double b_xr = 7.3898e-5 * crn_x_over_expm1(V - 3.3328, 5.1237);
    double t_xr = 1.0 / (a_xr + b_xr);
    double xrinf = 1.0 / (1.0 + exp((V + 14.1) / -6.5));
    double a_xs = 4e-5 * crn_x_over_1mexp(V - 19.9, 17.0);
    double b_xs = 3.5e-5 * crn_x_over_expm1(V - 19.9, 9.0);
    double t_xs = 0.5 / (a_xs + b_xs);
    double xsinf = 1.0 / sqrt(1.0 + exp((V - 19.9) / -12.7));
    /* tau_d = (1 - e^{-x/6.24}) / (0.035 x (1 + e^{-x/6.24})), x = V + 10 */
    double xd = V + 10.0;
    double t_d = 1.0 / (0.035 * crn_x_over_1mexp(xd, 6.24) * (1.0 + exp(-xd / 6.24)));
    double dinf = 1.0 / (1.0 + exp(-xd / 8.0));
    double t_f = 9.0 / (0.0197 * exp(-0.0337 * 0.0337 * xd * xd) + 0.02);
    double finf = 1.0 / (1.0 + exp((V + 28.0) / 6.9));
    double fcainf = 1.0 / (1.0 + Cai / 0.00035);
    double t_fca = 2.0;
    double Fn = 1e-12 * CRN_VREL * Irel
              - 5e-13 / CRN_F * (0.5 * CRN_CM * c.ICaL - 0.2 * CRN_CM * c.INaCa);
    double su = 1.0 / (1.0 + exp(-(Fn - 3.4175e-13) / 13.67e-16));
    double uinf = su;
    double t_u = 8.0;
    double vinf = 1.0 - 1.0 / (1.0 + exp(-(Fn - 6.835e-14) / 13.67e-16));
    double t_v = 1.91 + 2.09 * su;
    double winf = 1.0 - 1.0 / (1.0 + exp(-(V - 40.0) / 17.0));
    /* tau_w = 6 (1 - e^{-x/5}) / ((1 + 0.3 e^{-x/5}) x), x = V - 7.9 */
    double xw = V - 7.9;
    double t_w = 6.0 / (crn_x_over_1mexp(xw, 5.0) * (1.0 + 0.3 * exp(-xw / 5.0)));

    /* forward Euler for the concentrations */
    y[0] += dt * dNai;
    y[1] += dt * dKi;
    y[2] += dt * dCai;
    y[3] += dt * dCaup;
    y[4] += dt * dCarel;
    /* Rush-Larsen for the gates */
    y[5] = rl(y[5], am / (am + bm), 1.0 / (am + bm), dt);
    y[6] = rl(y[6], ah / (ah + bh), 1.0 / (ah + bh), dt);
    y[7] = rl(y[7], aj / (aj + bj), 1.0 / (aj + bj), dt);
    y[8] = rl(y[8], oainf, t_oa, dt);
    y[9] = rl(y[9], oiinf, t_oi, dt);
    y[10] = rl(y[10], uainf, t_ua, dt);
    y[11] = rl(y[11], uiinf, t_ui, dt);
    y[12] = rl(y[12], xrinf, t_xr, dt);
    y[13] = rl(y[13], xsinf, t_xs, dt);
    y[14] = rl(y[14], dinf, t_d, dt);
    y[15] = rl(y[15], finf, t_f, dt);
    y[16] = rl(y[16], fcainf, t_fca, dt);
    y[17] = rl(y[17], uinf, t_u, dt);
    y[18] = rl(y[18], vinf, t_v, dt);
    y[19] = rl(y[19], winf, t_w, dt);

    /* I_ion(V^k, u^{k+1}) */
    crn_currents_at(g, V, y, &c);
    *iion = crn_sum(&c);
}

/* number of states (excluding V) and parameters per model kind
 * kind 0: no ionic current (diffusion only), 1: Mitchell-Schaeffer, 2: TTP06,
 * 3: Courtemanche-Ramirez-Nattel */
int orc_ionic_nstates(int kind)
{
    return kind == 1 ? 1 : kind == 2 ? TT_NS : kind == 3 ? CRN_NS : 0;
}
int orc_ionic_nparams(int kind)
{
    return kind == 1 ? MS_NPAR : kind == 2 ? TT_NPAR : kind == 3 ? CRN_NPAR : 0;
}

void orc_ionic_defaults(int kind, double *params)
{
    if (kind == 1) memcpy(params, MS_DEFAULT, sizeof(MS_DEFAULT));
    if (kind == 2) memcpy(params, TT_DEFAULT, sizeof(TT_DEFAULT));
    if (kind == 3) memcpy(params, CRN_DEFAULT, sizeof(CRN_DEFAULT));
}

/* rest state: V0 and u0 (SoA, u[s*n + i]) */
void orc_ionic_init(int kind, const double *params, int64_t n, double *V, double *u)
{
    for (int64_t i = 0; i < n; ++i) {
        if (kind == 1) { V[i] = params[5]; u[i] = 1.0; }
        else if (kind == 2) {
            V[i] = TT_V0;
            for (int s = 0; s < TT_NS; ++s) u[(int64_t)s * n + i] = TT_INIT[s];
        } else if (kind == 3) {
            V[i] = CRN_V0;
            for (int s = 0; s < CRN_NS; ++s) u[(int64_t)s * n + i] = CRN_INIT[s];
        } else V[i] = 0.0;
    }
}

/* one ionic step at every node: u <- u^{k+1}; iion <- I_ion(V^k,u^{k+1}) / Cm */
void orc_ionic_step(int kind, const double *params, int64_t n, double dt,
                    const double *V, double *u, double *iion)
{
#pragma omp parallel for schedule(static) if (n > 20000)
    for (int64_t i = 0; i < n; ++i) {
        if (kind == 1) {
            ms_point(params, dt, V[i], &u[i], &iion[i]);
        } else if (kind == 2) {
            double y[TT_NS];
            for (int s = 0; s < TT_NS; ++s) y[s] = u[(int64_t)s * n + i];
            tt_point(params, dt, V[i], y, &iion[i]);
            for (int s = 0; s < TT_NS; ++s) u[(int64_t)s * n + i] = y[s];
        } else if (kind == 3) {
            double y[CRN_NS];
            for (int s = 0; s < CRN_NS; ++s) y[s] = u[(int64_t)s * n + i];
            crn_point(params, dt, V[i], y, &iion[i]);
            for (int s = 0; s < CRN_NS; ++s) u[(int64_t)s * n + i] = y[s];
        } else {
            iion[i] = 0.0;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Time stepping.  One step k -> k+1 (Eq. 2 and the A, b definitions):        */
/*   u^{k+1} = ionic update from (V^k, u^k); I_ion = Cm * I(V^k, u^{k+1});   */
/*   b = chi M (Cm V^k + dt (I_stim^k - I_ion + src)) - (1-theta) dt K V^k;   */
/*   A = chi Cm M + theta dt K;  A V^{k+1} = b by Jacobi-PCG from x0.        */
/* Reading: Eq. (2) prints "+ (1-theta) dt K" on the right while the b       */
/* definition prints "- (1-theta) dt K V^k"; the minus sign is the theta-    */
/* method and is used here.                                                  */
/* Stimulus s is active at step k iff round(start/dt) <= k < round((start+   */
/* duration)/dt); overlapping stimuli add.                                   */
/* LAT_i = t^{k+1} the first time V_i^{k+1} > 0; LRT_i = t^{k+1} the first   */
/* time after activation that V_i^{k+1} < -70 with V_i^{k+1} < V_i^k.        */
/* tissue = {chi, cm, theta, dt}; isolver = {rel_mode, max_iter, warm_start} */
/* (warm_start 0: x0 = V^k; 1: x0 = 2 V^k - V^{k-1}); solver = {atol, rtol}. */
/* extra_src (nullable) holds one extra per-node source per step, in uA/mm^2 */
/* like I_stim: row (k - k0) of an [n_steps][n] array (manufactured-solution */
/* tests use it).                                                            */
/* iters_out[k] receives the PCG iteration count (-1: not converged).        */
/* ------------------------------------------------------------------------ */
int orc_steps(int64_t n, const int64_t *row_ptr, const int32_t *col,
              const double *Mv, const double *Kv, const double *tissue,
              int ionic_kind, const double *ionic_params,
              int n_stim, const int64_t *stim_off, const int32_t *stim_idx,
              const double *stim_par, const double *solver, const int32_t *isolver,
              double *V, double *Vprev, double *u, double *lat, double *lrt,
              int64_t k0, int64_t n_steps, int64_t out_every, double *v_out,
              int32_t *iters_out, const double *extra_src)
{
    const double chi = tissue[0], cm = tissue[1], theta = tissue[2], dt = tissue[3];
    int64_t nnz = row_ptr[n];
    double *A = malloc(sizeof(double) * (size_t)nnz);
    for (int64_t s = 0; s < nnz; ++s) A[s] = chi * cm * Mv[s] + theta * dt * Kv[s];
    double *iion = malloc(sizeof(double) * (size_t)n);
    double *istim = malloc(sizeof(double) * (size_t)n);
    double *w = malloc(sizeof(double) * (size_t)n);
    double *mw = malloc(sizeof(double) * (size_t)n);
    double *kv = malloc(sizeof(double) * (size_t)n);
    double *b = malloc(sizeof(double) * (size_t)n);
    double *x = malloc(sizeof(double) * (size_t)n);
    int64_t n_out = 0;
    int rc = 0;

    for (int64_t k = k0; k < k0 + n_steps; ++k) {
        orc_ionic_step(ionic_kind, ionic_params, n, dt, V, u, iion);

        memset(istim, 0, sizeof(double) * (size_t)n);
        for (int s = 0; s < n_stim; ++s) {
            int64_t ks = llround(stim_par[3 * s] / dt);
            int64_t ke = llround((stim_par[3 * s] + stim_par[3 * s + 1]) / dt);
            if (k >= ks && k < ke)
                for (int64_t q = stim_off[s]; q < stim_off[s + 1]; ++q)
                    istim[stim_idx[q]] += stim_par[3 * s + 2];
        }
        for (int64_t i = 0; i < n; ++i) {
            double src = extra_src ? extra_src[(k - k0) * n + i] : 0.0;
            w[i] = cm * V[i] + dt * (istim[i] - cm * iion[i] + src);
        }
        orc_spmv(n, row_ptr, col, Mv, w, mw);
        orc_spmv(n, row_ptr, col, Kv, V, kv);
        for (int64_t i = 0; i < n; ++i) b[i] = chi * mw[i] - (1.0 - theta) * dt * kv[i];

        for (int64_t i = 0; i < n; ++i)
            x[i] = isolver[2] == 1 ? 2.0 * V[i] - Vprev[i] : V[i];
        int it = orc_pcg(n, row_ptr, col, A, b, x, solver[0], solver[1], isolver[0],
                         isolver[1], NULL);
        if (iters_out) iters_out[k - k0] = it;
        if (it < 0) rc = 1;

        double t1 = (double)(k + 1) * dt;
        for (int64_t i = 0; i < n; ++i) {
            if (lat && isinf(lat[i]) && x[i] > 0.0) lat[i] = t1;
            if (lrt && lat && !isinf(lat[i]) && lat[i] < t1 && isinf(lrt[i])
                && x[i] < -70.0 && x[i] < V[i])
                lrt[i] = t1;
            Vprev[i] = V[i];
            V[i] = x[i];
        }
        if (v_out && out_every > 0 && (k + 1 - k0) % out_every == 0) {
            memcpy(v_out + n_out * n, V, sizeof(double) * (size_t)n);
            ++n_out;
        }
    }
    free(A); free(iion); free(istim); free(w); free(mw); free(kv); free(b); free(x);
    return rc;
}

/* OpenMP thread control for timing runs */
#include <omp.h>
void orc_set_threads(int t) { if (t > 0) omp_set_num_threads(t); }
int orc_get_threads(void) { return omp_get_max_threads(); }
