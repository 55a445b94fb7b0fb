/*
 * rkl_oracle.c -- serial FP64 reference for one RKL2 super-step of
 * field-aligned (anisotropic) thermal conduction.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker that the HIP path is
 * compared against.  Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark may load it; the product path never does.  It shares no
 * code, header, table or helper with the HIP library.
 *
 * Source: Vaidya, Prasad, Mignone, Sharma & Rickler (2017), "Scalable explicit
 * implementation of anisotropic diffusion with Runge-Kutta-Legendre
 * super-time-stepping" (arXiv:1702.05487).
 *
 * What is computed (all FP64, no blocking, no fusion):
 *   - the conductive flux at every cell face: harmonic blend of the classical
 *     field-aligned flux and the saturated flux (Sec. 2, Eqs. Fc, Fclass,
 *     Fsat; the perpendicular term that Sec. 2 calls straightforward to add),
 *     with the transverse temperature gradients either averaged or limited
 *     with the monotonized-central limiter (Sec. 3.4 and Appendix B);
 *   - the conservative second-order divergence of that flux (Sec. 3, the
 *     finite-difference formula under Eq. scalar_diffusion);
 *   - the explicit parabolic step (Sec. 3.1, Eq. dt_exp, HD diffusivity);
 *   - the number of RKL2 stages from the super-step (Sec. 3.3, Eq. RKL-s,
 *     rounded up as stated at the start of Sec. 4.1);
 *   - the RKL2 coefficients and stage scheme (Appendix A, Eq. rkl2scheme and
 *     the coefficient formulas that follow it).
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   face temperature = mean of the two cells; conductivities and the
 *   saturated flux use max(T_face, 0); the face field direction is the
 *   normalised sum of the two cell unit vectors (zero when that sum is
 *   shorter than 1e-12); the limited transverse gradient at a face is
 *   MC(MC(a1,a2), MC(a3,a4)) over the one-sided differences of the two cells,
 *   the unlimited one is their mean; the saturated flux takes q at the face
 *   temperature (central) or, in the upwind form that Sec. 3 names without
 *   giving it, at the temperature of the cell the classical face flux
 *   leaves, with the full face flux vector's magnitude in the harmonic
 *   blend either way; c_iso = sqrt(T)
 *   (p = rho T in code units); the stage operator is evaluated on each
 *   stage's own temperature and tau*M(Y0) is computed once and reused;
 *   each axis is periodic, outflow (ghost cells repeat the edge cell's T
 *   and b) or fixed (ghost temperatures given by the caller and held over
 *   the super-step, as the Gaussian test of Sec. 4.1.1 takes its edge values
 *   from the exact solution; b repeats the edge cell's).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no fast-math), so every
 * a*b+c rounds twice, exactly as written.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of the cell loops.  Every cell's value is computed on its own
 * from inputs that the loop does not write, so the result is the same bits
 * for any thread count; the default is one thread (serial). */
static int orc_threads = 1;

void orc_set_threads(int n) { orc_threads = n < 1 ? 1 : n; }

int orc_get_threads(void)
{
#ifdef _OPENMP
    return orc_threads;
#else
    return 1;
#endif
}

/* Grid and physics parameters.  Layout of every field: [n2][n1][n0], axis 0
 * fastest.  b is three such arrays back to back (component-major). */
typedef struct {
    int ndim;           /* 1, 2 or 3; axes >= ndim must have n = 1 */
    int n[3];           /* cells per axis */
    double h[3];        /* cell widths */
    int limiter;        /* 0: mean of the four one-sided differences, 1: MC */
    int saturation;     /* 0: classical flux only, 1: harmonic blend with q of
                           the face temperature, 2: the same with q of the
                           upwind cell (the upwind treatment of the
                           saturated term named in Sec. 3) */
    double phi;         /* saturation uncertainty factor (Eq. Fsat) */
    double kappa0;      /* kappa_par = kappa0 * T^kappa_exp */
    double kappa_exp;
    double kperp_ratio; /* kappa_perp = kperp_ratio * kappa_par */
    double rho;         /* frozen density */
    double gamma;       /* ratio of specific heats */
    double cp;          /* parabolic Courant number, <= 1/2 */
    int boundary[3];    /* per axis: 0 periodic, 1 outflow (the cells beyond
                           an edge repeat the edge cell: zero-gradient ghosts),
                           2 fixed (ghost temperatures from ghost[d]) */
    /* fixed axis d: ghost[d][0] and ghost[d][1] are the temperatures beyond
     * the low and the high edge, one layer each, of (n_b + 2) x (n_a + 2)
     * values (a < b the other two axes), index (j_b + 1) (n_a + 2) + j_a + 1
     * for transverse position (j_a, j_b), j in [-1, n].  A position beyond
     * the edges of several fixed axes takes the layer of the lowest of them;
     * a transverse index is wrapped on a periodic axis, clamped to [0, n-1]
     * on an outflow axis and to [-1, n] on a fixed one; every position
     * beyond an edge (however far) takes that edge's layer. */
    const double *ghost[3][2];
} orc_grid;

static long ncell(const orc_grid *g) { return (long)g->n[0] * g->n[1] * g->n[2]; }

/* index of cell (c[0], c[1], c[2]): wrapped on periodic axes, clamped to
 * the edge cell on outflow axes */
static long cell_index(const orc_grid *g, const int c[3])
{
    int w[3];
    for (int d = 0; d < 3; ++d) {
        if (g->boundary[d]) {
            w[d] = c[d] < 0 ? 0 : (c[d] >= g->n[d] ? g->n[d] - 1 : c[d]);
        } else {
            int m = c[d] % g->n[d];
            w[d] = m < 0 ? m + g->n[d] : m;
        }
    }
    return ((long)w[2] * g->n[1] + w[1]) * g->n[0] + w[0];
}

/* temperature at position c: a ghost value where c lies beyond an edge of a
 * fixed axis, else the (wrapped or clamped) cell's */
static double temp_at(const orc_grid *g, const double *T, const int c[3])
{
    for (int d = 0; d < 3; ++d) {
        if (g->boundary[d] != 2 || (c[d] >= 0 && c[d] < g->n[d])) continue;
        const int side = c[d] >= g->n[d];
        int t[2], k = 0;
        for (int e = 0; e < 3; ++e) {
            if (e == d) continue;
            const int n = g->n[e];
            int v = c[e];
            if (g->boundary[e] == 0) {
                v %= n;
                if (v < 0) v += n;
            } else {
                const int lo = g->boundary[e] == 2 ? -1 : 0, hi = g->boundary[e] == 2 ? n : n - 1;
                v = v < lo ? lo : (v > hi ? hi : v);
            }
            t[k++] = v;
        }
        int na = 0;
        for (int e = 0; e < 3; ++e)
            if (e != d) { na = g->n[e]; break; }
        return g->ghost[d][side][(long)(t[1] + 1) * (na + 2) + (t[0] + 1)];
    }
    return T[cell_index(g, c)];
}

static double value_at(const orc_grid *g, const double *f, const int c[3], int d, int shift)
{
    int q[3] = {c[0], c[1], c[2]};
    q[d] += shift;
    return temp_at(g, f, q);
}

/* Parallel conductivity kappa0 * T^kappa_exp with T clipped at zero. */
static double kappa_par(const orc_grid *g, double T)
{
    double t = T > 0.0 ? T : 0.0;
    if (g->kappa_exp == 0.0) return g->kappa0;
    if (g->kappa_exp == 2.5) return g->kappa0 * (t * t * sqrt(t));
    return g->kappa0 * pow(t, g->kappa_exp);
}

/* Monotonized-central limiter of two slopes: minmod(2a, 2b, (a+b)/2). */
double orc_mc(double a, double b)
{
    if (a * b <= 0.0) return 0.0;
    double m = fabs(a + b) * 0.5;
    double ta = 2.0 * fabs(a), tb = 2.0 * fabs(b);
    if (ta < m) m = ta;
    if (tb < m) m = tb;
    return a > 0.0 ? m : -m;
}

/*
 * Component d of the conductive flux through the face between cell c and its
 * +e_d neighbour (Eqs. Fc, Fclass, Fsat plus the perpendicular term).
 */
static double face_flux(const orc_grid *g, const double *T, const double *b,
                        const int c[3], int d)
{
    const long N = ncell(g);
    int r[3] = {c[0], c[1], c[2]};
    r[d] += 1;
    const long iL = cell_index(g, c), iR = cell_index(g, r);
    const double TL = temp_at(g, T, c), TR = temp_at(g, T, r);

    /* temperature and conductivities at the face */
    const double Tf = 0.5 * (TL + TR);
    const double kpar = kappa_par(g, Tf);
    const double kperp = g->kperp_ratio * kpar;

    /* field direction at the face */
    double bf[3], nb2 = 0.0;
    for (int e = 0; e < 3; ++e) {
        bf[e] = b[e * N + iL] + b[e * N + iR];
        nb2 += bf[e] * bf[e];
    }
    const double nb = sqrt(nb2);
    for (int e = 0; e < 3; ++e) bf[e] = nb < 1e-12 ? 0.0 : bf[e] / nb;

    /* temperature gradient at the face: normal component is face-native,
     * the two transverse components come from one-sided differences in the
     * two cells that share the face (Appendix B) */
    double G[3];
    for (int e = 0; e < 3; ++e) {
        if (e == d) {
            G[e] = (TR - TL) / g->h[d];
            continue;
        }
        const double he = g->h[e];
        double a1 = (TL - value_at(g, T, c, e, -1)) / he;
        double a2 = (value_at(g, T, c, e, +1) - TL) / he;
        double a3 = (TR - value_at(g, T, r, e, -1)) / he;
        double a4 = (value_at(g, T, r, e, +1) - TR) / he;
        if (g->limiter)
            G[e] = orc_mc(orc_mc(a1, a2), orc_mc(a3, a4));
        else
            G[e] = 0.25 * (a1 + a2 + a3 + a4);
    }

    /* classical flux vector  F = -[kperp G + (kpar - kperp) b (b.G)] */
    const double bG = bf[0] * G[0] + bf[1] * G[1] + bf[2] * G[2];
    double F[3];
    for (int e = 0; e < 3; ++e)
        F[e] = -(kperp * G[e] + (kpar - kperp) * bf[e] * bG);

    if (!g->saturation) return F[d];

    /* saturated flux q = 5 phi rho c_iso^3 with c_iso = sqrt(T), blended
     * harmonically with the magnitude of the classical flux (Eq. Fc).  T is
     * the face temperature, or in the upwind form the temperature of the
     * cell that the heat leaves through this face: L when the classical flux
     * points from L to R (F_d > 0), else R. */
    double Tq = Tf;
    if (g->saturation == 2) Tq = F[d] > 0.0 ? TL : TR;
    const double t = Tq > 0.0 ? Tq : 0.0;
    const double q = 5.0 * g->phi * g->rho * (t * sqrt(t));
    const double Fm = sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2]);
    if (q == 0.0) return 0.0;
    return q / (q + Fm) * F[d];
}

/* Component d of the flux through the +e_d face of cell (i, j, k), as used
 * by the divergence below (exported for the pins of the face algebra). */
double orc_face_flux(const orc_grid *g, const double *T, const double *b, int i, int j, int k, int d)
{
    const int c[3] = {i, j, k};
    return face_flux(g, T, b, c, d);
}

/*
 * out = (gamma-1)/rho * ( -div F_c(T) ), the conservative second-order
 * difference of the face fluxes (Sec. 3).  With rho*eps = rho T/(gamma-1)
 * this is dT/dt of Eq. scalar_diffusion.
 */
void orc_flux_div(const orc_grid *g, const double *T, const double *b, double *out)
{
    const double fac = (g->gamma - 1.0) / g->rho;
#pragma omp parallel for collapse(2) num_threads(orc_threads) schedule(static) if (orc_threads > 1)
    for (int k = 0; k < g->n[2]; ++k)
        for (int j = 0; j < g->n[1]; ++j)
            for (int i = 0; i < g->n[0]; ++i) {
                const int c[3] = {i, j, k};
                double div = 0.0;
                for (int d = 0; d < g->ndim; ++d) {
                    int l[3] = {i, j, k};
                    l[d] -= 1;
                    const double Fp = face_flux(g, T, b, c, d);
                    const double Fm = face_flux(g, T, b, l, d);
                    div += (Fp - Fm) / g->h[d];
                }
                out[cell_index(g, c)] = fac * (-div);
            }
}

/*
 * Explicit parabolic step (Eq. dt_exp) with the HD diffusivity
 * chi = kappa_par (gamma-1)/rho in every direction, maximised over cells.
 * Returns +inf when the maximum is zero.
 */
double orc_dt_par(const orc_grid *g, const double *T)
{
    double inv_h2 = 0.0;
    for (int d = 0; d < g->ndim; ++d) inv_h2 += 1.0 / (g->h[d] * g->h[d]);
    const double fac = (g->gamma - 1.0) / g->rho;
    double lam = 0.0;
    const long N = ncell(g);
    for (long i = 0; i < N; ++i) {
        const double v = fac * kappa_par(g, T[i]) * inv_h2;
        if (v > lam) lam = v;
    }
    if (lam == 0.0) return INFINITY;
    return g->cp / lam;
}

/*
 * Number of RKL2 stages for r = dt_hyp/dt_par: the real root of
 * r = (s^2 + s - 2)/4 (Eq. RKL-s), then s -> 1 + floor(s) (Sec. 4.1).
 */
int orc_stages(double r)
{
    const double s_real = (-1.0 + sqrt(9.0 + 16.0 * r)) / 2.0;
    return 1 + (int)floor(s_real);
}

/*
 * RKL2 coefficients for an s-stage super-step (Appendix A).  Arrays are
 * indexed by stage j = 0..s; entries that the scheme does not use are 0.
 *   b_j = (j^2+j-2)/(2j(j+1)) for j > 2, b_0 = b_1 = b_2 = 1/3, a_j = 1 - b_j
 *   w1 = 4/(s^2+s-2)
 *   mut_1 = b_1 w1
 *   mu_j = (2j-1)/j * b_j/b_{j-1},  nu_j = -(j-1)/j * b_j/b_{j-2}
 *   mut_j = mu_j w1,  gt_j = -a_{j-1} mut_j          (2 <= j <= s)
 */
void orc_coeffs(int s, double *w1_out, double *mu, double *nu, double *mut, double *gt)
{
    /* RKL2 needs s >= 2 (w1 = 4/(s^2+s-2)); the callers check it.  The b_j
     * table always holds j = 0..2 so that b_1 is defined whatever s is. */
    const int nb = s < 2 ? 2 : s;
    double *bj = (double *)malloc(sizeof(double) * (nb + 1));
    for (int j = 0; j <= nb; ++j) {
        if (j <= 2) bj[j] = 1.0 / 3.0;
        else bj[j] = ((double)j * j + j - 2.0) / (2.0 * j * (j + 1.0));
    }
    const double w1 = 4.0 / ((double)s * s + s - 2.0);
    for (int j = 0; j <= s; ++j) mu[j] = nu[j] = mut[j] = gt[j] = 0.0;
    mut[1] = bj[1] * w1;
    for (int j = 2; j <= s; ++j) {
        mu[j] = (2.0 * j - 1.0) / j * bj[j] / bj[j - 1];
        nu[j] = -(j - 1.0) / j * bj[j] / bj[j - 2];
        mut[j] = mu[j] * w1;
        gt[j] = -(1.0 - bj[j - 1]) * mut[j];
    }
    *w1_out = w1;
    free(bj);
}

/*
 * s stages of RKL2 over a super-step tau (Eq. rkl2scheme); T holds Y_0 on
 * entry and Y_s on return.  M is the flux-divergence operator above,
 * evaluated on each stage's own temperature.
 */
void orc_rkl2_fixed(const orc_grid *g, double *T, const double *b, int s, double tau)
{
    const long N = ncell(g);
    double *mu = malloc(sizeof(double) * (s + 1)), *nu = malloc(sizeof(double) * (s + 1));
    double *mut = malloc(sizeof(double) * (s + 1)), *gt = malloc(sizeof(double) * (s + 1));
    double w1;
    orc_coeffs(s, &w1, mu, nu, mut, gt);

    double *Y0 = malloc(sizeof(double) * N), *MY0 = malloc(sizeof(double) * N);
    double *Yjm2 = malloc(sizeof(double) * N), *Yjm1 = malloc(sizeof(double) * N);
    double *Yj = malloc(sizeof(double) * N), *L = malloc(sizeof(double) * N);

    memcpy(Y0, T, sizeof(double) * N);
    orc_flux_div(g, Y0, b, L);
    for (long i = 0; i < N; ++i) MY0[i] = tau * L[i];
    for (long i = 0; i < N; ++i) Yjm1[i] = Y0[i] + mut[1] * MY0[i];
    memcpy(Yjm2, Y0, sizeof(double) * N);

    for (int j = 2; j <= s; ++j) {
        orc_flux_div(g, Yjm1, b, L);
        for (long i = 0; i < N; ++i)
            Yj[i] = mu[j] * Yjm1[i] + nu[j] * Yjm2[i] + (1.0 - mu[j] - nu[j]) * Y0[i]
                  + mut[j] * tau * L[i] + gt[j] * MY0[i];
        double *t = Yjm2; Yjm2 = Yjm1; Yjm1 = Yj; Yj = t;
    }
    memcpy(T, Yjm1, sizeof(double) * N);

    free(mu); free(nu); free(mut); free(gt);
    free(Y0); free(MY0); free(Yjm2); free(Yjm1); free(Yj); free(L);
}

/*
 * One RKL2 super-step of length dt_hyp: dt_par from T, s from the ratio,
 * then the stages.  Returns s; *dt_par_out receives dt_par.
 */
int orc_superstep(const orc_grid *g, double *T, const double *b, double dt_hyp, double *dt_par_out)
{
    const double dtp = orc_dt_par(g, T);
    const double r = isinf(dtp) ? 0.0 : dt_hyp / dtp;
    const int s = orc_stages(r);
    if (dt_par_out) *dt_par_out = dtp;
    orc_rkl2_fixed(g, T, b, s, dt_hyp);
    return s;
}

/* Sub-cycling (Sec. 2.3, explicit methods; Sec. 5.2 case (b)): the conduction
 * operator applied N_sub times with a stable step, here
 * N_sub = ceil(dt_hyp / dt_par) with dt_par of Eq. dt_exp taken from T at the
 * start, each sub-step forward Euler  T <- T + tau (gamma-1)/rho (-div F_c(T))
 * with tau = dt_hyp / N_sub <= dt_par.  Returns N_sub (0 when dt_hyp = 0 or
 * there is no conduction: T unchanged; -1 if N_sub would exceed max_sub). */
long orc_subcycle(const orc_grid *g, double *T, const double *b, double dt_hyp, long max_sub)
{
    const double dtp = orc_dt_par(g, T);
    if (!(dt_hyp > 0.0) || isinf(dtp)) return 0;
    const double q = ceil(dt_hyp / dtp);
    if (!(q <= (double)max_sub)) return -1;
    const long nsub = (long)q;
    const double tau = dt_hyp / (double)nsub;
    const long N = ncell(g);
    double *L = malloc(sizeof(double) * N);
    for (long k = 0; k < nsub; ++k) {
        orc_flux_div(g, T, b, L);
        for (long i = 0; i < N; ++i) T[i] = T[i] + tau * L[i];
    }
    free(L);
    return nsub;
}

/*
 * RKL1, the first-order Legendre scheme (Sec. 3.3): stability polynomial
 * R_s(z) = P_s(1 + w1 z) (a_s = 0, b_s = 1 in Eq. stabpara) with
 * w1 = 2/(s^2+s), and dt_hyp = dt_par (s^2+s)/2 (Eq. RKL-s).  The stages
 * follow the Legendre recursion (Eq. recLegP) with x = 1 + w1 tau M:
 *   Y_1 = Y_0 + w1 tau M(Y_0)
 *   Y_j = (2j-1)/j (Y_{j-1} + w1 tau M(Y_{j-1})) - (j-1)/j Y_{j-2},  j >= 2,
 * so that Y_s = P_s(1 + w1 tau M) Y_0 for linear M; M is evaluated on each
 * stage's own temperature.  s = 1 is one forward-Euler step.
 */
int orc_stages_rkl1(double r)
{
    const double s_real = (-1.0 + sqrt(1.0 + 8.0 * r)) / 2.0;
    return 1 + (int)floor(s_real);
}

void orc_rkl1_fixed(const orc_grid *g, double *T, const double *b, int s, double tau)
{
    const long N = ncell(g);
    const double w1 = 2.0 / ((double)s * s + s);
    double *Yjm2 = malloc(sizeof(double) * N), *Yjm1 = malloc(sizeof(double) * N);
    double *Yj = malloc(sizeof(double) * N), *L = malloc(sizeof(double) * N);

    memcpy(Yjm2, T, sizeof(double) * N);
    orc_flux_div(g, Yjm2, b, L);
    for (long i = 0; i < N; ++i) Yjm1[i] = Yjm2[i] + w1 * tau * L[i];

    for (int j = 2; j <= s; ++j) {
        orc_flux_div(g, Yjm1, b, L);
        const double a = (2.0 * j - 1.0) / j, c = (j - 1.0) / j;
        for (long i = 0; i < N; ++i)
            Yj[i] = a * (Yjm1[i] + w1 * tau * L[i]) - c * Yjm2[i];
        double *t = Yjm2; Yjm2 = Yjm1; Yjm1 = Yj; Yj = t;
    }
    memcpy(T, Yjm1, sizeof(double) * N);
    free(Yjm2); free(Yjm1); free(Yj); free(L);
}

/* One RKL1 super-step of length dt_hyp: dt_par from T, s from the ratio
 * (rounded up as for RKL2), then the stages.  Returns s. */
int orc_superstep_rkl1(const orc_grid *g, double *T, const double *b, double dt_hyp, double *dt_par_out)
{
    const double dtp = orc_dt_par(g, T);
    const double r = isinf(dtp) ? 0.0 : dt_hyp / dtp;
    const int s = orc_stages_rkl1(r);
    if (dt_par_out) *dt_par_out = dtp;
    orc_rkl1_fixed(g, T, b, s, dt_hyp);
    return s;
}

/*
 * AAG super-time-stepping (Alexiades, Amiez & Gremaud 1996; Sec. 3.3): s
 * forward-Euler sub-steps with the damped Chebyshev sequence
 *   tau_j = dt_p / ((nu - 1) cos(pi (2j - 1) / (2s)) + 1 + nu),  j = 1..s,
 * whose sum is the gain of Eq. AAG-STS,
 *   dt_p s / (2 sqrt(nu)) [(1+sqrt(nu))^{2s} - (1-sqrt(nu))^{2s}]
 *                         / [(1+sqrt(nu))^{2s} + (1-sqrt(nu))^{2s}].
 * orc_aag_gain returns that bracket times s/(2 sqrt(nu)) (the sum over dt_p);
 * once (1+sqrt(nu))^{2s} is beyond the double range the bracket is 1 to
 * double precision ((1-sqrt(nu))^{2s} <= 1), and is taken as 1;
 * orc_aag_stages the smallest s whose gain reaches r = dt_hyp/dt_par;
 * orc_aag_superstep scales the sequence of that s to sum to dt_hyp (each
 * sub-step then stays within the sequence built on dt_par) and applies it.
 */
double orc_aag_gain(int s, double nu)
{
    const double q = sqrt(nu);
    const double a = pow(1.0 + q, 2.0 * s), c = pow(1.0 - q, 2.0 * s);
    if (isinf(a)) return s / (2.0 * q);
    return s / (2.0 * q) * ((a - c) / (a + c));   /* the bracket first: s/(2q) a may overflow */
}

int orc_aag_stages(double r, double nu, int smax)
{
    for (int s = 1; s <= smax; ++s)
        if (orc_aag_gain(s, nu) >= r) return s;
    return -1;
}

void orc_aag_taus(int s, double nu, double dt_p, double *tau)
{
    const double pi = 3.14159265358979323846;
    for (int j = 1; j <= s; ++j)
        tau[j - 1] = dt_p / ((nu - 1.0) * cos(pi * (2.0 * j - 1.0) / (2.0 * s)) + 1.0 + nu);
}

/* s AAG sub-steps whose sequence is scaled to sum to dt_hyp */
void orc_aag_fixed(const orc_grid *g, double *T, const double *b, int s, double nu, double dt_hyp)
{
    double *tau = malloc(sizeof(double) * s);
    orc_aag_taus(s, nu, 1.0, tau);
    double sum = 0.0;
    for (int j = 0; j < s; ++j) sum += tau[j];
    const long N = ncell(g);
    double *L = malloc(sizeof(double) * N);
    for (int j = 0; j < s; ++j) {
        const double t = tau[j] * (dt_hyp / sum);
        orc_flux_div(g, T, b, L);
        for (long i = 0; i < N; ++i) T[i] = T[i] + t * L[i];
    }
    free(L);
    free(tau);
}

int orc_aag_superstep(const orc_grid *g, double *T, const double *b, double dt_hyp, double nu, int smax)
{
    const double dtp = orc_dt_par(g, T);
    if (!(dt_hyp > 0.0) || isinf(dtp)) return 0;
    const int s = orc_aag_stages(dt_hyp / dtp, nu, smax);
    if (s < 0) return -1;
    orc_aag_fixed(g, T, b, s, nu, dt_hyp);
    return s;
}
