/*
 * eam_oracle.c -- plain, slow, FP64 reference for EAM free-energy switching.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant with the
 * HIP library; both sides read the same seeded inputs and nothing else.
 *
 * What it computes, in the paper's order and notation (arXiv 2201.04622):
 *   - H0 = KE + U with U an embedded-atom (EAM) potential        (Eq. H, Sec. bulk)
 *   - Einstein crystal U_E = sum 1/2 k |r - r0|^2, k = m w^2       (Eq. einstein)
 *   - Frenkel-Ladd blend H(l) = (1-l) H0 + l H_E                   (Eq. interp)
 *   - Reversible-scaling H(l) = KE + l U                           (Eq. H_rs)
 *   - work as the left-point sum  W = sum_k dl_k (dH/dl)(G(k dt))   (Eq. w_irr, discrete form)
 *   - lambda(tau) of the ti/spring switching (function 1 and 2) and of the RS scan
 *   - Langevin thermostat with the centre of mass held fixed (Sec. p_fl, "flying ice cube")
 * Readings where the paper is silent (tabulation, thermostat discretisation,
 * noise layout) are listed with the design notes; they are:
 *   tables  : natural cubic splines on uniform knots; interval m = floor(x/h)
 *             clamped to [0, n-2], t = x/h - m (the last cubic is continued past
 *             the end); a pair contributes only if r < r_cut.
 *   EAM     : U = sum_i F(rho_i) + 1/2 sum_{i!=j} phi(r_ij), rho_i = sum_{j!=i} rho(r_ij)
 *             (standard single-species form; the paper only names "EAM").
 *   images  : minimum image in an orthorhombic periodic box, positions unwrapped.
 *   thermostat : BAOAB splitting with gamma = 1/damp; with gamma = 0 it is the
 *             velocity-Verlet integrator the paper uses for its NVE check.
 *   switching: at step s the work increment uses dH/dl at x_s, then the step is
 *             propagated with lambda_{s+1}.
 *   noise   : Philox4x32-10 (Salmon et al., SC'11), key = (seed lo, seed hi),
 *             counter = (atom, step lo, stream, step hi); Box-Muller on
 *             u = (x+1)/2^32.  stream 0 = thermostat, 1 = initial velocities.
 *   fixed CM: the per-replica mean of the thermostat noise is removed, and the
 *             initial velocities have zero total momentum.
 *
 * Pins: every function here is checked by the tests against closed forms,
 * invariants, library routines or published values; the Philox bit stream
 * against the generator's published known-answer vectors.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* LAMMPS metal units (CODATA 2018 values). */
#define ORC_KB     8.617333262e-5   /* eV / K                         */
#define ORC_HBAR   6.582119569e-4   /* eV ps                          */
#define ORC_MVV2E  1.0364269e-4     /* eV per (amu A^2 / ps^2)        */

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_ENOMEM = 2, ORC_ETABLE = 4, ORC_EBOX = 8 };
enum { ORC_FL = 0, ORC_RS = 1, ORC_HH = 2, ORC_EIN_RS = 3 };

/* ------------------------------------------------------------------------ */
/* Natural cubic spline on a uniform grid (tabulated potential functions).    */
/* ------------------------------------------------------------------------ */

/* Coefficients of the natural cubic spline through y[0..n-1] at x_k = k h.
 * On interval m, with t = x/h - m in [0,1]:
 *   s = a + t (b + t (c + t d)),
 * a = y_m, b = y_{m+1} - y_m - h^2 (2 M_m + M_{m+1}) / 6,
 * c = h^2 M_m / 2, d = h^2 (M_{m+1} - M_m) / 6,
 * where M are the second derivatives: M_0 = M_{n-1} = 0 and
 * M_{k-1} + 4 M_k + M_{k+1} = 6 (y_{k+1} - 2 y_k + y_{k-1}) / h^2.
 * coef is [n-1][4].  Returns 0 or ORC_EINVAL / ORC_ENOMEM. */
int orc_spline_natural(int n, double h, const double* y, double* coef)
{
    if (n < 3 || !(h > 0.0)) return ORC_EINVAL;
    double* M = (double*)calloc((size_t)n, sizeof(double));
    double* cp = (double*)calloc((size_t)n, sizeof(double));
    double* dp = (double*)calloc((size_t)n, sizeof(double));
    if (!M || !cp || !dp) { free(M); free(cp); free(dp); return ORC_ENOMEM; }
    /* Thomas algorithm on the interior unknowns M_1 .. M_{n-2}. */
    for (int k = 1; k <= n - 2; ++k) {
        double rhs = 6.0 * (y[k + 1] - 2.0 * y[k] + y[k - 1]) / (h * h);
        double sub = (k > 1) ? 1.0 : 0.0;
        double denom = 4.0 - sub * cp[k - 1];
        cp[k] = 1.0 / denom;                      /* super-diagonal is 1 */
        dp[k] = (rhs - sub * dp[k - 1]) / denom;
    }
    M[0] = 0.0;
    M[n - 1] = 0.0;
    for (int k = n - 2; k >= 1; --k)
        M[k] = dp[k] - cp[k] * ((k + 1 <= n - 2) ? M[k + 1] : 0.0);
    for (int m = 0; m < n - 1; ++m) {
        coef[4 * m + 0] = y[m];
        coef[4 * m + 1] = y[m + 1] - y[m] - h * h * (2.0 * M[m] + M[m + 1]) / 6.0;
        coef[4 * m + 2] = h * h * M[m] / 2.0;
        coef[4 * m + 3] = h * h * (M[m + 1] - M[m]) / 6.0;
    }
    free(M); free(cp); free(dp);
    return ORC_OK;
}

/* Interval index and local coordinate for x on the uniform grid. */
static int orc_interval(int n, double h, double x, double* t)
{
    double p = x / h;
    int m = (int)floor(p);
    if (m < 0) m = 0;
    if (m > n - 2) m = n - 2;
    *t = p - (double)m;
    return m;
}

/* Spline value and derivative at x. */
double orc_spline_eval(int n, double h, const double* coef, double x, double* dydx)
{
    double t;
    int m = orc_interval(n, h, x, &t);
    const double* c = coef + 4 * m;
    if (dydx) *dydx = (c[1] + t * (2.0 * c[2] + 3.0 * t * c[3])) / h;
    return c[0] + t * (c[1] + t * (c[2] + t * c[3]));
}

/* ------------------------------------------------------------------------ */
/* Tabulated EAM potential                                                   */
/* ------------------------------------------------------------------------ */
typedef struct orc_pot {
    int n_r, n_rho;
    double r_cut, h_r, rho_max, h_rho;
    double *phi, *rho, *F;            /* spline coefficients [n-1][4] */
} orc_pot;

void orc_pot_free(orc_pot* p)
{
    if (!p) return;
    free(p->phi); free(p->rho); free(p->F); free(p);
}

/* Knots: phi and rho at r_k = k r_cut/(n_r-1); F at rho_k = k rho_max/(n_rho-1). */
orc_pot* orc_pot_create(int n_r, double r_cut, const double* phi_knots, const double* rho_knots,
                        int n_rho, double rho_max, const double* F_knots)
{
    if (n_r < 3 || n_rho < 3 || !(r_cut > 0.0) || !(rho_max > 0.0)) return NULL;
    orc_pot* p = (orc_pot*)calloc(1, sizeof(orc_pot));
    if (!p) return NULL;
    p->n_r = n_r; p->n_rho = n_rho;
    p->r_cut = r_cut; p->h_r = r_cut / (n_r - 1);
    p->rho_max = rho_max; p->h_rho = rho_max / (n_rho - 1);
    p->phi = (double*)malloc(sizeof(double) * 4 * (size_t)(n_r - 1));
    p->rho = (double*)malloc(sizeof(double) * 4 * (size_t)(n_r - 1));
    p->F = (double*)malloc(sizeof(double) * 4 * (size_t)(n_rho - 1));
    if (!p->phi || !p->rho || !p->F ||
        orc_spline_natural(n_r, p->h_r, phi_knots, p->phi) ||
        orc_spline_natural(n_r, p->h_r, rho_knots, p->rho) ||
        orc_spline_natural(n_rho, p->h_rho, F_knots, p->F)) {
        orc_pot_free(p);
        return NULL;
    }
    return p;
}

/* Copy out the interval coefficients, [3][n-1][4] for (phi, rho, F). */
void orc_pot_coefficients(const orc_pot* p, double* phi, double* rho, double* F)
{
    memcpy(phi, p->phi, sizeof(double) * 4 * (size_t)(p->n_r - 1));
    memcpy(rho, p->rho, sizeof(double) * 4 * (size_t)(p->n_r - 1));
    memcpy(F, p->F, sizeof(double) * 4 * (size_t)(p->n_rho - 1));
}

/* Minimum-image separation d = x_i - x_j in an orthorhombic box. */
static void orc_min_image(const double* xi, const double* xj, const double* L, double* d)
{
    for (int c = 0; c < 3; ++c) {
        double s = xi[c] - xj[c];
        d[c] = s - L[c] * nearbyint(s / L[c]);
    }
}

/* Optional neighbour candidates: for atom i, nb[i*cap .. i*cap+cnt[i]) lists
 * every j != i that was within r_cut + skin when the list was made.  NULL nb
 * means "all j" (brute force). */
typedef struct orc_nlist {
    int cap;
    int* cnt;
    int* nb;
    double* xref;     /* [N][3] positions at build time */
    double skin;
} orc_nlist;

static int orc_nlist_build(orc_nlist* nl, int N, const double* x, const double* L, double r_cut)
{
    double rl2 = (r_cut + nl->skin) * (r_cut + nl->skin);
    for (int i = 0; i < N; ++i) {
        int c = 0;
        for (int j = 0; j < N; ++j) {
            if (j == i) continue;
            double d[3];
            orc_min_image(x + 3 * i, x + 3 * j, L, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 < rl2) {
                if (c >= nl->cap) return ORC_EINVAL;
                nl->nb[(size_t)i * nl->cap + c++] = j;
            }
        }
        nl->cnt[i] = c;
    }
    memcpy(nl->xref, x, sizeof(double) * 3 * (size_t)N);
    return ORC_OK;
}

static int orc_nlist_stale(const orc_nlist* nl, int N, const double* x)
{
    double lim = 0.25 * nl->skin * nl->skin;   /* (skin/2)^2 */
    for (int i = 0; i < N; ++i) {
        double d0 = x[3 * i] - nl->xref[3 * i], d1 = x[3 * i + 1] - nl->xref[3 * i + 1],
               d2 = x[3 * i + 2] - nl->xref[3 * i + 2];
        if (d0 * d0 + d1 * d1 + d2 * d2 > lim) return 1;
    }
    return 0;
}

/* EAM energy and forces (Eq. H with U = EAM).
 *   rho_i = sum_{j != i, r_ij < r_cut} rho(r_ij)
 *   U     = sum_i F(rho_i) + 1/2 sum_i sum_{j != i, r_ij < r_cut} phi(r_ij)
 *   f_i   = - sum_{j != i} [phi'(r) + (F'(rho_i) + F'(rho_j)) rho'(r)] (x_i - x_j)/r
 * x, f are [N][3].  Optional outputs (may be NULL): e_atom[N] = F(rho_i) +
 * 1/2 sum_j phi, rho[N], Fp[N].  Returns ORC_ETABLE if some rho_i > rho_max
 * (the values are still computed by continuing the last cubic). */
static int orc_eam_impl(const orc_pot* p, int N, const double* x, const double* L, const orc_nlist* nl,
                        double* f, double* U, double* e_atom, double* rho_out, double* Fp_out, double* vir)
{
    int status = ORC_OK;
    double rc2 = p->r_cut * p->r_cut;
    double* rho = (double*)calloc((size_t)N, sizeof(double));
    double* Fp = (double*)calloc((size_t)N, sizeof(double));
    if (!rho || !Fp) { free(rho); free(Fp); return ORC_ENOMEM; }
    double Usum = 0.0;
    /* density */
    for (int i = 0; i < N; ++i) {
        int cnt = nl ? nl->cnt[i] : N;
        double s = 0.0;
        for (int q = 0; q < cnt; ++q) {
            int j = nl ? nl->nb[(size_t)i * nl->cap + q] : q;
            if (j == i) continue;
            double d[3];
            orc_min_image(x + 3 * i, x + 3 * j, L, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 >= rc2) continue;
            s += orc_spline_eval(p->n_r, p->h_r, p->rho, sqrt(r2), NULL);
        }
        rho[i] = s;
        if (s > p->rho_max) status |= ORC_ETABLE;
        double dF;
        double Fi = orc_spline_eval(p->n_rho, p->h_rho, p->F, s, &dF);
        Fp[i] = dF;
        if (e_atom) e_atom[i] = Fi;
        Usum += Fi;
    }
    /* pair energy and forces; virial sum_{i<j} d_a f_a = (1/2) sum_i sum_j d_a f_a with
     * d = x_i - x_j and f the force on i due to j */
    double w[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < N; ++i) {
        int cnt = nl ? nl->cnt[i] : N;
        double fi[3] = {0.0, 0.0, 0.0};
        double ei = 0.0;
        for (int q = 0; q < cnt; ++q) {
            int j = nl ? nl->nb[(size_t)i * nl->cap + q] : q;
            if (j == i) continue;
            double d[3];
            orc_min_image(x + 3 * i, x + 3 * j, L, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 >= rc2) continue;
            double r = sqrt(r2);
            double dphi, drho;
            double ph = orc_spline_eval(p->n_r, p->h_r, p->phi, r, &dphi);
            (void)orc_spline_eval(p->n_r, p->h_r, p->rho, r, &drho);
            double g = dphi + (Fp[i] + Fp[j]) * drho;   /* dU/dr_ij */
            for (int c = 0; c < 3; ++c) {
                fi[c] -= g * d[c] / r;
                w[c] -= 0.5 * g * d[c] * d[c] / r;
            }
            ei += 0.5 * ph;
        }
        if (f) for (int c = 0; c < 3; ++c) f[3 * i + c] = fi[c];
        if (e_atom) e_atom[i] += ei;
        Usum += ei;
    }
    if (U) *U = Usum;
    if (vir) for (int c = 0; c < 3; ++c) vir[c] = w[c];
    if (rho_out) memcpy(rho_out, rho, sizeof(double) * (size_t)N);
    if (Fp_out) memcpy(Fp_out, Fp, sizeof(double) * (size_t)N);
    free(rho); free(Fp);
    return status;
}

int orc_eam(const orc_pot* p, int N, const double* x, const double* L,
            double* f, double* U, double* e_atom, double* rho, double* Fp)
{
    for (int c = 0; c < 3; ++c)
        if (!(L[c] > 2.0 * p->r_cut)) return ORC_EBOX;   /* one image at most */
    return orc_eam_impl(p, N, x, L, NULL, f, U, e_atom, rho, Fp, NULL);
}

/* Diagonal of the pressure tensor of an EAM configuration (the quantity the
 * paper holds at zero with its barostat before the Frenkel--Ladd runs):
 * P_aa = (sum_i m v_ia^2 + W_aa) / V with the pair virial W_aa = sum_{i<j}
 * (x_i - x_j)_a f_ij,a of the central EAM pair forces.  v may be NULL (the
 * configurational part only).  Output P[3] in eV/A^3. */
int orc_pressure(const orc_pot* p, int N, const double* x, const double* v, double mass, const double* L,
                 double* P)
{
    for (int c = 0; c < 3; ++c)
        if (!(L[c] > 2.0 * p->r_cut)) return ORC_EBOX;
    double w[3];
    int st = orc_eam_impl(p, N, x, L, NULL, NULL, NULL, NULL, NULL, NULL, w);
    const double V = L[0] * L[1] * L[2];
    for (int c = 0; c < 3; ++c) {
        double k2 = 0.0;
        if (v) for (int i = 0; i < N; ++i) k2 += v[3 * i + c] * v[3 * i + c];
        P[c] = (mass * ORC_MVV2E * k2 + w[c]) / V;
    }
    return st;
}

/* Force on, energy of, and density of one atom i (for sampled checks of very
 * large systems): O(N) for rho_i plus O(N) per neighbour for rho_j. */
int orc_eam_atom(const orc_pot* p, int N, const double* x, const double* L, int i,
                 double* f3, double* e_atom, double* rho_i_out)
{
    double rc2 = p->r_cut * p->r_cut;
    int status = ORC_OK;
    /* rho_j for arbitrary j by a direct sum */
#define ORC_RHO_OF(jj, out)                                                             \
    do {                                                                               \
        double s_ = 0.0;                                                               \
        for (int k_ = 0; k_ < N; ++k_) {                                               \
            if (k_ == (jj)) continue;                                                  \
            double d_[3];                                                              \
            orc_min_image(x + 3 * (jj), x + 3 * k_, L, d_);                            \
            double r2_ = d_[0] * d_[0] + d_[1] * d_[1] + d_[2] * d_[2];                \
            if (r2_ < rc2) s_ += orc_spline_eval(p->n_r, p->h_r, p->rho, sqrt(r2_), NULL); \
        }                                                                              \
        (out) = s_;                                                                    \
    } while (0)
    double rho_i;
    ORC_RHO_OF(i, rho_i);
    if (rho_i > p->rho_max) status |= ORC_ETABLE;
    double Fpi;
    double Fi = orc_spline_eval(p->n_rho, p->h_rho, p->F, rho_i, &Fpi);
    double fi[3] = {0.0, 0.0, 0.0}, ei = Fi;
    for (int j = 0; j < N; ++j) {
        if (j == i) continue;
        double d[3];
        orc_min_image(x + 3 * i, x + 3 * j, L, d);
        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (r2 >= rc2) continue;
        double rho_j, Fpj;
        ORC_RHO_OF(j, rho_j);
        (void)orc_spline_eval(p->n_rho, p->h_rho, p->F, rho_j, &Fpj);
        double r = sqrt(r2), dphi, drho;
        double ph = orc_spline_eval(p->n_r, p->h_r, p->phi, r, &dphi);
        (void)orc_spline_eval(p->n_r, p->h_r, p->rho, r, &drho);
        double g = dphi + (Fpi + Fpj) * drho;
        for (int c = 0; c < 3; ++c) fi[c] -= g * d[c] / r;
        ei += 0.5 * ph;
    }
#undef ORC_RHO_OF
    for (int c = 0; c < 3; ++c) f3[c] = fi[c];
    if (e_atom) *e_atom = ei;
    if (rho_i_out) *rho_i_out = rho_i;
    return status;
}

/* ------------------------------------------------------------------------ */
/* Counter-based noise: Philox4x32-10 and Box-Muller                         */
/* ------------------------------------------------------------------------ */

/* Philox4x32 with 10 rounds as published by Salmon, Moraes, Dror and Shaw
 * (SC'11): each round multiplies words 0 and 2 by the two round multipliers,
 * mixes the high halves with the other words and the key, and the key is
 * advanced by the two Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Three standard normal deviates for (seed, atom, step, stream). */
void orc_gauss3(uint64_t seed, uint32_t atom, int64_t step, uint32_t stream, double z[3])
{
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    uint64_t st = (uint64_t)step;
    uint32_t ctr[4] = {atom, (uint32_t)(st & 0xFFFFFFFFu), stream, (uint32_t)(st >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    const double two32inv = 1.0 / 4294967296.0;
    const double twopi = 6.283185307179586476925286766559;
    double u0 = ((double)w[0] + 1.0) * two32inv;
    double u1 = ((double)w[1] + 1.0) * two32inv;
    double u2 = ((double)w[2] + 1.0) * two32inv;
    double u3 = ((double)w[3] + 1.0) * two32inv;
    double r0 = sqrt(-2.0 * log(u0));
    double r1 = sqrt(-2.0 * log(u2));
    z[0] = r0 * cos(twopi * u1);
    z[1] = r0 * sin(twopi * u1);
    z[2] = r1 * cos(twopi * u3);
}

/* ------------------------------------------------------------------------ */
/* Switching functions and schedules (Sec. fl_lammps, Sec. RS in LAMMPS)     */
/* ------------------------------------------------------------------------ */

/* ti/spring lambda(tau): function 1 is linear, function 2 the 9th-order
 * polynomial with vanishing slope at both ends. */
double orc_lambda_fl(int function, double tau)
{
    if (function == 1) return tau;
    double t5 = tau * tau * tau * tau * tau;
    return t5 * (70.0 * tau * tau * tau * tau - 315.0 * tau * tau * tau + 540.0 * tau * tau
                 - 420.0 * tau + 126.0);
}

/* RS lambda(tau) = 1 / (1 + tau (1/lambda_f - 1)), i.e. T = T0/lambda linear in tau. */
double orc_lambda_rs(double lambda_f, double tau)
{
    return 1.0 / (1.0 + tau * (1.0 / lambda_f - 1.0));
}

/* Lambda table of length S+1 for the five ti/spring phases (FL, HH):
 * [n_eq at 0][n_sw forward 0->1][n_hold at 1][n_sw backward 1->0][n_hold2 at 0],
 * tau = (elapsed switching steps)/n_sw.  For RS (and EIN_RS):
 * [n_eq at 1][n_sw forward 1->lambda_f][n_hold at lambda_f][n_sw backward][n_hold2 at 1],
 * the backward branch being the time reverse of the forward one. */
int orc_schedule(int mode, int function, double lambda_f, int n_eq, int n_sw, int n_hold,
                 int n_hold2, double* lam)
{
    if (n_eq < 0 || n_sw < 1 || n_hold < 0 || n_hold2 < 0) return ORC_EINVAL;
    int rs = (mode == ORC_RS || mode == ORC_EIN_RS);
    int S = n_eq + 2 * n_sw + n_hold + n_hold2;
    int s = 0;
    double lo = rs ? 1.0 : 0.0;
    for (; s <= n_eq; ++s) lam[s] = lo;
    for (int q = 1; q <= n_sw; ++q, ++s) {
        double tau = (double)q / (double)n_sw;
        lam[s] = rs ? orc_lambda_rs(lambda_f, tau) : orc_lambda_fl(function, tau);
    }
    for (int q = 1; q <= n_hold; ++q, ++s) lam[s] = lam[n_eq + n_sw];
    int b0 = n_eq + n_sw + n_hold;
    for (int q = 1; q <= n_sw; ++q, ++s) {
        double tau = 1.0 - (double)q / (double)n_sw;   /* time reverse */
        lam[s] = rs ? orc_lambda_rs(lambda_f, tau) : orc_lambda_fl(function, tau);
    }
    (void)b0;
    for (int q = 1; q <= n_hold2; ++q, ++s) lam[s] = lo;
    return (s == S + 1) ? ORC_OK : ORC_EINVAL;
}

/* ------------------------------------------------------------------------ */
/* Langevin switching run                                                    */
/* ------------------------------------------------------------------------ */
typedef struct orc_params {
    int mode;            /* ORC_FL, ORC_RS, ORC_HH, ORC_EIN_RS                    */
    int fix_com;         /* remove the mean thermostat noise                      */
    double T;            /* K                                                     */
    double gamma;        /* 1/ps (1/damp); 0 gives velocity Verlet                */
    double dt;           /* ps                                                    */
    double mass;         /* amu                                                   */
    double k;            /* eV/A^2: Einstein spring (FL, EIN_RS) or k1 (HH)       */
    double k2;           /* eV/A^2: HH final spring                               */
    uint64_t seed;
    double skin;         /* > 0: use a Verlet candidate list with this skin       */
    int nlist_cap;
} orc_params;

/* Potential-energy components at x: U_EAM (with forces fE), and the spring sum
 * S2 = sum_i s_i |x_i - x0_i|^2 with per-atom spring scales s_i (1 when ks is
 * NULL): atom i's spring is k s_i, its force -k s_i (x_i - x0_i) (Sec. on
 * multi-species springs: one spring constant per group of atoms). */
typedef struct orc_comp {
    double U_eam;
    double S2;
    double* f_eam;       /* [N][3] */
    const double* ks;    /* [N] spring scales or NULL */
} orc_comp;

static int orc_components(const orc_pot* p, const orc_params* P, int N, const double* x,
                          const double* x0, const double* L, const orc_nlist* nl, orc_comp* c)
{
    int st = ORC_OK;
    if (P->mode == ORC_FL || P->mode == ORC_RS) {
        st = orc_eam_impl(p, N, x, L, nl, c->f_eam, &c->U_eam, NULL, NULL, NULL, NULL);
    } else {
        c->U_eam = 0.0;
        memset(c->f_eam, 0, sizeof(double) * 3 * (size_t)N);
    }
    double s2 = 0.0;
    for (int i = 0; i < N; ++i) {
        double d2 = 0.0;
        for (int q = 0; q < 3; ++q) d2 += (x[3 * i + q] - x0[3 * i + q]) * (x[3 * i + q] - x0[3 * i + q]);
        s2 += (c->ks ? c->ks[i] : 1.0) * d2;
    }
    c->S2 = s2;
    return st;
}

/* dH/dlambda at a fixed phase point for each mode (kinetic energy does not
 * depend on lambda):
 *   FL     (Eq. w_irr2): U_E - U_EAM
 *   RS     (Eq. w_irr_rs): U_EAM
 *   HH     : U_E(k2) - U_E(k1)
 *   EIN_RS : U_E(k)                                                          */
static double orc_dHdl(const orc_params* P, const orc_comp* c)
{
    switch (P->mode) {
    case ORC_FL: return 0.5 * P->k * c->S2 - c->U_eam;
    case ORC_RS: return c->U_eam;
    case ORC_HH: return 0.5 * (P->k2 - P->k) * c->S2;
    default:     return 0.5 * P->k * c->S2;
    }
}

/* Total force on atom component at lambda. */
static double orc_force(const orc_params* P, const orc_comp* c, const double* x, const double* x0,
                        int idx, double lam)
{
    double dx = (x[idx] - x0[idx]) * (c->ks ? c->ks[idx / 3] : 1.0);   /* s_i (x - x0) */
    switch (P->mode) {
    case ORC_FL: return (1.0 - lam) * c->f_eam[idx] + lam * (-P->k * dx);
    case ORC_RS: return lam * c->f_eam[idx];
    case ORC_HH: return -((1.0 - lam) * P->k + lam * P->k2) * dx;
    default:     return lam * (-P->k * dx);
    }
}

/* Potential energy at lambda (for conservation checks). */
static double orc_upot(const orc_params* P, const orc_comp* c, double lam)
{
    double UE = 0.5 * P->k * c->S2;
    switch (P->mode) {
    case ORC_FL: return (1.0 - lam) * c->U_eam + lam * UE;
    case ORC_RS: return lam * c->U_eam;
    case ORC_HH: return 0.5 * ((1.0 - lam) * P->k + lam * P->k2) * c->S2;
    default:     return lam * UE;
    }
}

/* Initial velocities: v = sqrt(kT/m) * z(stream 1, step 0); with fix_com the
 * mean is removed so the centre of mass starts at rest. */
void orc_init_velocities(const orc_params* P, int N, double* v)
{
    double sig = sqrt(ORC_KB * P->T / (P->mass * ORC_MVV2E));
    double mean[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < N; ++i) {
        double z[3];
        orc_gauss3(P->seed, (uint32_t)i, 0, 1u, z);
        for (int c = 0; c < 3; ++c) { v[3 * i + c] = sig * z[c]; mean[c] += v[3 * i + c]; }
    }
    if (P->fix_com) {
        for (int c = 0; c < 3; ++c) mean[c] /= (double)N;
        for (int i = 0; i < N; ++i)
            for (int c = 0; c < 3; ++c) v[3 * i + c] -= mean[c];
    }
}

/* Run S steps from (x, v) with the lambda table lam[0..S] (global step index
 * of the first step: step0, which keys the noise).  Per step s:
 *   1. W += (lam[s+1] - lam[s]) dH/dl(x_s);  dHdl_out[s], W_out[s] recorded
 *   2. v += dt/(2m) F(x_s; lam[s+1])               (B)
 *   3. x += dt/2 v                                 (A)
 *   4. v  = c1 v + sqrt((1-c1^2) kT/m) (xi - <xi>)   (O), c1 = exp(-gamma dt)
 *   5. x += dt/2 v                                 (A)
 *   6. v += dt/(2m) F(x_{s+1}; lam[s+1])           (B)
 * W0 is the work carried in.  Optional e_out[S]: total energy KE + U(lam[s+1])
 * after the step.  Returns a status bit set (ORC_ETABLE possible). */
int orc_run(const orc_pot* p, const orc_params* P, int N, const double* x0, const double* L,
            double* x, double* v, int S, const double* lam, int64_t step0, double W0,
            double* dHdl_out, double* W_out, double* e_out, const double* ks)
{
    if (N < 1 || S < 0) return ORC_EINVAL;
    if (P->mode == ORC_FL || P->mode == ORC_RS) {
        double rl = p->r_cut + (P->skin > 0.0 ? P->skin : 0.0);
        for (int c = 0; c < 3; ++c)
            if (!(L[c] > 2.0 * rl)) return ORC_EBOX;
    }
    int status = ORC_OK;
    orc_comp comp;
    comp.ks = ks;
    comp.f_eam = (double*)calloc(3 * (size_t)N, sizeof(double));
    double* xi = (double*)calloc(3 * (size_t)N, sizeof(double));
    orc_nlist nl;
    orc_nlist* nlp = NULL;
    memset(&nl, 0, sizeof(nl));
    if (!comp.f_eam || !xi) { free(comp.f_eam); free(xi); return ORC_ENOMEM; }
    if (P->skin > 0.0 && (P->mode == ORC_FL || P->mode == ORC_RS)) {
        nl.cap = P->nlist_cap > 0 ? P->nlist_cap : 512;
        nl.skin = P->skin;
        nl.cnt = (int*)calloc((size_t)N, sizeof(int));
        nl.nb = (int*)calloc((size_t)N * nl.cap, sizeof(int));
        nl.xref = (double*)calloc(3 * (size_t)N, sizeof(double));
        if (!nl.cnt || !nl.nb || !nl.xref) { status = ORC_ENOMEM; goto done; }
        if (orc_nlist_build(&nl, N, x, L, p->r_cut)) { status = ORC_EINVAL; goto done; }
        nlp = &nl;
    }
    const double inv_m = 1.0 / (P->mass * ORC_MVV2E);          /* (A/ps^2) per (eV/A) */
    const double c1 = exp(-P->gamma * P->dt);
    const double c2 = sqrt((1.0 - c1 * c1) * ORC_KB * P->T * inv_m);
    status |= orc_components(p, P, N, x, x0, L, nlp, &comp);
    double W = W0;
    for (int s = 0; s < S; ++s) {
        double dHdl = orc_dHdl(P, &comp);
        W += (lam[s + 1] - lam[s]) * dHdl;
        if (dHdl_out) dHdl_out[s] = dHdl;
        if (W_out) W_out[s] = W;
        double ln = lam[s + 1];
        for (int q = 0; q < 3 * N; ++q) v[q] += 0.5 * P->dt * inv_m * orc_force(P, &comp, x, x0, q, ln);
        for (int q = 0; q < 3 * N; ++q) x[q] += 0.5 * P->dt * v[q];
        double mean[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < N; ++i) {
            orc_gauss3(P->seed, (uint32_t)i, step0 + s, 0u, xi + 3 * i);
            for (int c = 0; c < 3; ++c) mean[c] += xi[3 * i + c];
        }
        for (int c = 0; c < 3; ++c) mean[c] = P->fix_com ? mean[c] / (double)N : 0.0;
        for (int i = 0; i < N; ++i)
            for (int c = 0; c < 3; ++c)
                v[3 * i + c] = c1 * v[3 * i + c] + c2 * (xi[3 * i + c] - mean[c]);
        for (int q = 0; q < 3 * N; ++q) x[q] += 0.5 * P->dt * v[q];
        if (nlp && orc_nlist_stale(nlp, N, x)) {
            if (orc_nlist_build(nlp, N, x, L, p->r_cut)) { status |= ORC_EINVAL; goto done; }
        }
        status |= orc_components(p, P, N, x, x0, L, nlp, &comp);
        for (int q = 0; q < 3 * N; ++q) v[q] += 0.5 * P->dt * inv_m * orc_force(P, &comp, x, x0, q, ln);
        if (e_out) {
            double ke = 0.0;
            for (int q = 0; q < 3 * N; ++q) ke += v[q] * v[q];
            e_out[s] = 0.5 * P->mass * ORC_MVV2E * ke + orc_upot(P, &comp, ln);
        }
    }
done:
    free(comp.f_eam); free(xi);
    free(nl.cnt); free(nl.nb); free(nl.xref);
    return status;
}

/* ------------------------------------------------------------------------ */
/* dU/dtheta for the knot values theta = (phi_k, rho_k, F_k)                  */
/* ------------------------------------------------------------------------ */

/* U is linear in the interval coefficients of phi and F and, through rho_i,
 * depends on those of rho.  With B = (1, t, t^2, t^3) of each evaluation:
 *   dU/dc_phi[m]  = 1/2 sum_{i != j, r < rc, m(r)=m} B(t)
 *   dU/dc_F[m]    = sum_{i, m(rho_i)=m} B(t)
 *   dU/dc_rho[m]  = sum_i F'(rho_i) sum_{j, m(r_ij)=m} B(t)
 * and the knot gradient is the transpose of the linear knot -> coefficient map,
 * obtained here by brute force: dU/dy_k = <dU/dc, coef(spline of e_k)>.
 * g_out is [3][n] in the order (phi, rho, F).  Note phi and rho share n_r. */
int orc_adjoint_theta(const orc_pot* p, int N, const double* x, const double* L, double* g_out)
{
    int nr = p->n_r, nf = p->n_rho;
    double rc2 = p->r_cut * p->r_cut;
    double* gphi = (double*)calloc(4 * (size_t)(nr - 1), sizeof(double));
    double* grho = (double*)calloc(4 * (size_t)(nr - 1), sizeof(double));
    double* gF = (double*)calloc(4 * (size_t)(nf - 1), sizeof(double));
    double* rho = (double*)calloc((size_t)N, sizeof(double));
    double* Fp = (double*)calloc((size_t)N, sizeof(double));
    int nmax = nr > nf ? nr : nf;
    double* e = (double*)calloc((size_t)nmax, sizeof(double));
    double* ce = (double*)calloc(4 * (size_t)(nmax - 1), sizeof(double));
    int status = ORC_OK;
    if (!gphi || !grho || !gF || !rho || !Fp || !e || !ce) { status = ORC_ENOMEM; goto out; }
    status = orc_eam_impl(p, N, x, L, NULL, NULL, NULL, NULL, rho, Fp, NULL);
    for (int i = 0; i < N; ++i) {
        double t;
        int m = orc_interval(nf, p->h_rho, rho[i], &t);
        gF[4 * m + 0] += 1.0; gF[4 * m + 1] += t; gF[4 * m + 2] += t * t; gF[4 * m + 3] += t * t * t;
        for (int j = 0; j < N; ++j) {
            if (j == i) continue;
            double d[3];
            orc_min_image(x + 3 * i, x + 3 * j, L, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 >= rc2) continue;
            int mr = orc_interval(nr, p->h_r, sqrt(r2), &t);
            double B[4] = {1.0, t, t * t, t * t * t};
            for (int q = 0; q < 4; ++q) {
                gphi[4 * mr + q] += 0.5 * B[q];
                grho[4 * mr + q] += Fp[i] * B[q];
            }
        }
    }
    /* transpose through the cardinal splines */
    for (int fn = 0; fn < 3; ++fn) {
        int n = (fn == 2) ? nf : nr;
        double h = (fn == 2) ? p->h_rho : p->h_r;
        const double* g = (fn == 0) ? gphi : (fn == 1) ? grho : gF;
        for (int k = 0; k < n; ++k) {
            memset(e, 0, sizeof(double) * (size_t)n);
            e[k] = 1.0;
            orc_spline_natural(n, h, e, ce);
            double s = 0.0;
            for (int q = 0; q < 4 * (n - 1); ++q) s += g[q] * ce[q];
            g_out[(size_t)fn * nr + k] = s;
        }
    }
out:
    free(gphi); free(grho); free(gF); free(rho); free(Fp); free(e); free(ce);
    return status;
}
