/*
 * mgfr_oracle.c -- plain, slow FP64 CPU reference of the f(R) field solve.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the parity reference for the HIP
 * library: only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no code, header, table or helper with the
 * GPU path; it is unblocked and unfused on purpose so that it can be read
 * against the paper (Puchwein, Baldi & Springel 2013, "Modified
 * Gravity-GADGET") line by line.  Built plainly it is single-threaded; built
 * with -fopenmp the loops whose iterations are independent (the cells of one
 * colour of a red-black sweep, operator and transfer evaluations, max-norm
 * reductions) run on several threads with bitwise the same results, since no
 * floating-point sum changes its order.
 *
 * Units and form.  Positions are comoving Mpc/h, the cell side h = L/N is
 * comoving.  The paper's discrete field equation (Sec. 3.2, Eq.
 * u_discrete_field_eq) is written in physical units; multiplying it by a^2
 * and using 8 pi G rho_bar = 3 H0^2 Omega_m a^-3 and R_bar = 3 H0^2 C(a)
 * (Sec. 2, background curvature of flat LCDM) gives the dimensionless form
 * used throughout:
 *
 *   L_c(u) = (1/h^2) sum_nb 1/2 (e^{u_nb} + e^{u_c}) (u_nb - u_c)
 *            - beta C (1 - e^{-u_c/(n+1)})
 *   f_c    = beta Omega_m a^-3 delta_c
 *   beta   = a^2 (H0/c)^2 / |fbar_R(a)|,  C(a) = Omega_m a^-3 + 4 Omega_L
 *
 * which is the paper's operator and source times a^2 (an exact rescaling: the
 * relative residual is unchanged).  For n = 1 the curvature term is the
 * paper's Eq. dR_fR; for general n it follows from the large-curvature
 * relation f_R ~ R^-(n+1) (Sec. 2, Eq. fR-R,n_relation).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_C_OVER_H0 2997.92458   /* c/H0 in Mpc/h */
#define OR_C_KMS 299792.458       /* c in km/s */
#define OR_MAX_HIST 512

typedef struct {
    double box;      /* comoving box side, Mpc/h */
    double a;        /* scale factor */
    double omega_m, omega_l;
    double fr0_abs;  /* |fbar_R0| */
    int n;           /* Hu-Sawicki exponent */
    int mesh;        /* N, mesh cells per side (power of two >= 8) */
    double tol;      /* relative max-norm residual threshold */
    int pre_smooth, post_smooth, coarse_sweeps, max_vcycles;
    int prolong;     /* 0 = linear (gradient-based) reconstruction, 1 = straight injection */
    double max_du;   /* limit on |Newton step| per update; <= 0: no limit */
} or_params;

typedef struct {
    int vcycles;
    int status;      /* 0 converged, 1 not converged, -3 non-finite */
    double res0, res, scale;
    double res_hist[OR_MAX_HIST];
} or_stats;

/* Threads used by the OpenMP build (n > 0 sets them); 1 for the plain build. */
int or_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* max of two magnitudes with NaN winning (a NaN residual must not be hidden) */
static double nanmax(double a, double b)
{
    if (a != a || b != b) return NAN;
    return a > b ? a : b;
}

/* ---------------------------------------------------------------- background */

/* Sec. 2: R_bar(a) = 3 m^2 (a^-3 + 4 Omega_L/Omega_m) with m^2 = H0^2 Omega_m,
 * and fbar_R(a) = fbar_R0 (R_bar0 / R_bar(a))^(n+1) (Eq. fR_mean for n = 1,
 * Eq. fR-R,n_relation for general n).  Returns |fbar_R(a)|, beta and C. */
void or_background(const or_params *p, double *fbar, double *beta, double *C)
{
    double r = 4.0 * p->omega_l / p->omega_m;
    double a3 = 1.0 / (p->a * p->a * p->a);
    double fb = p->fr0_abs * pow((1.0 + r) / (a3 + r), p->n + 1);
    *fbar = fb;
    *C = p->omega_m * a3 + 4.0 * p->omega_l;
    *beta = p->a * p->a / (OR_C_OVER_H0 * OR_C_OVER_H0) / fb;
}

/* ------------------------------------------------------------ mass assignment */

static long wrapi(long i, long N) { long r = i % N; return r < 0 ? r + N : r; }

/* Sec. 3.1: cloud-in-cell.  Each particle is a cube of one cell side; cell
 * (i,j,k) covers [ih,(i+1)h) per axis, centre (i+1/2)h; the weights are the
 * overlap volumes.  Periodic.  mass == NULL means unit masses. */
void or_cic_assign(int N, double box, int64_t np, const float *pos,
                   const double *mass, double *m)
{
    double h = box / N;
    memset(m, 0, sizeof(double) * (size_t)N * N * N);
    for (int64_t p = 0; p < np; ++p) {
        long i0[3];
        double t[3];
        for (int d = 0; d < 3; ++d) {
            double xi = (double)pos[3 * p + d] / h - 0.5;
            double fl = floor(xi);
            t[d] = xi - fl;
            i0[d] = (long)fl;
        }
        double mp = mass ? mass[p] : 1.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int c = 0; c < 2; ++c) {
                    double w = (a ? t[0] : 1.0 - t[0]) * (b ? t[1] : 1.0 - t[1]) *
                               (c ? t[2] : 1.0 - t[2]);
                    long ii = wrapi(i0[0] + a, N), jj = wrapi(i0[1] + b, N), kk = wrapi(i0[2] + c, N);
                    m[(ii * N + jj) * N + kk] += w * mp;
                }
    }
}

/* delta = m / m_bar - 1 with m_bar the mean assigned cell mass. */
void or_delta(int N, const double *m, double *delta)
{
    size_t n3 = (size_t)N * N * N;
    double s = 0.0;
    for (size_t c = 0; c < n3; ++c) s += m[c];
    double mbar = s / (double)n3;
    for (size_t c = 0; c < n3; ++c) delta[c] = m[c] / mbar - 1.0;
}

/* Source term (Sec. 3.2, f_ijk) in the dimensionless form: beta Omega_m a^-3 delta. */
void or_source(const or_params *p, const double *delta, double *f)
{
    double fb, beta, C;
    or_background(p, &fb, &beta, &C);
    size_t n3 = (size_t)p->mesh * p->mesh * p->mesh;
    double s = beta * p->omega_m / (p->a * p->a * p->a);
#pragma omp parallel for
    for (size_t c = 0; c < n3; ++c) f[c] = s * delta[c];
}

/* Initial guess from the screened limit (Sec. 2, Eqs. fR_field_eq and
 * dR_fR): where the Laplacian of f_R is negligible the field equation reduces
 * to the local balance dR = 8 pi G d rho, which in the dimensionless variable
 * u = ln(f_R / fbar_R) reads exp(-u/(n+1)) = 1 + Omega_m a^-3 delta / C(a).
 * Only overdense cells take this value (the balance describes screened
 * regions); the others start at u = 0. */
void or_screened_guess(const or_params *p, const double *delta, double *u)
{
    double fb, beta, C;
    or_background(p, &fb, &beta, &C);
    size_t n3 = (size_t)p->mesh * p->mesh * p->mesh;
    double s = p->omega_m / (p->a * p->a * p->a) / C;
#pragma omp parallel for
    for (size_t c = 0; c < n3; ++c) {
        double d = delta[c] > 0.0 ? delta[c] : 0.0;
        u[c] = -(double)(p->n + 1) * log1p(s * d);
    }
}

/* Effective mass density of Sec. 3.4 (Eq. effective_density) in units of the
 * mean matter density: drho_eff / rho_bar = delta/3 - dR / (24 pi G rho_bar)
 * with dR = R_bar (e^{-u/(n+1)} - 1) (Eq. dR_fR and its general-n form),
 * R_bar = 3 H0^2 C(a) and 8 pi G rho_bar = 3 H0^2 Omega_m a^-3, i.e.
 * delta_eff = delta/3 - C expm1(-u/(n+1)) / (3 Omega_m a^-3). */
void or_effective_density(const or_params *p, const double *delta, const double *u, double *out)
{
    double fb, beta, C;
    or_background(p, &fb, &beta, &C);
    size_t n3 = (size_t)p->mesh * p->mesh * p->mesh;
    double om = p->omega_m / (p->a * p->a * p->a);
    double q = 1.0 / (p->n + 1);
#pragma omp parallel for
    for (size_t c = 0; c < n3; ++c) out[c] = delta[c] / 3.0 - C * expm1(-q * u[c]) / (3.0 * om);
}

/* ---------------------------------------------------------------- operator */

#define IDX(i, j, k) ((((size_t)(i)) * N + (j)) * N + (k))

/* L_c and its derivative with respect to u_c at one cell.  The flux-form
 * Laplacian of e^u uses face coefficients b = (e^{u_a} + e^{u_b})/2 times the
 * differences of u (Sec. 3.2); the derivative includes the u_c dependence of
 * the face coefficients (Newton's d L / d u of Eq. iterative_correction). */
static double op_cell(const double *u, int N, int i, int j, int k, double ih2,
                      double bC, double q, double *J)
{
    int ip = (i + 1) % N, im = (i + N - 1) % N;
    int jp = (j + 1) % N, jm = (j + N - 1) % N;
    int kp = (k + 1) % N, km = (k + N - 1) % N;
    double uc = u[IDX(i, j, k)];
    double nb[6] = {u[IDX(ip, j, k)], u[IDX(im, j, k)], u[IDX(i, jp, k)],
                    u[IDX(i, jm, k)], u[IDX(i, j, kp)], u[IDX(i, j, km)]};
    double ec = exp(uc);
    double lap = 0.0, dlap = 0.0;
    for (int s = 0; s < 6; ++s) {
        double en = exp(nb[s]);
        lap += 0.5 * (en + ec) * (nb[s] - uc);
        dlap += 0.5 * (ec * (nb[s] - uc - 1.0) - en);
    }
    /* 1 - e^{-q u} via expm1: no cancellation for small |u| */
    double em = expm1(-q * uc);
    if (J) *J = ih2 * dlap - bC * q * (1.0 + em);
    return ih2 * lap + bC * em;
}

/* Apply L to the whole periodic N^3 mesh with cell side h. */
void or_apply_L(int N, double h, double bC, int n, const double *u, double *L)
{
    double ih2 = 1.0 / (h * h), q = 1.0 / (n + 1);
#pragma omp parallel for
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
            for (int k = 0; k < N; ++k) L[IDX(i, j, k)] = op_cell(u, N, i, j, k, ih2, bC, q, NULL);
}

/* d L_c / d u_c at every cell (used by tests to check the derivative). */
void or_apply_J(int N, double h, double bC, int n, const double *u, double *Jout)
{
    double ih2 = 1.0 / (h * h), q = 1.0 / (n + 1);
#pragma omp parallel for
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
            for (int k = 0; k < N; ++k) op_cell(u, N, i, j, k, ih2, bC, q, &Jout[IDX(i, j, k)]);
}

/* Max-norm of f - L(u). */
double or_residual_max(int N, double h, double bC, int n, const double *u, const double *f)
{
    double ih2 = 1.0 / (h * h), q = 1.0 / (n + 1), mx = 0.0;
#pragma omp parallel
    {
        double lm = 0.0;
#pragma omp for
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j)
                for (int k = 0; k < N; ++k) {
                    double r = fabs(f[IDX(i, j, k)] - op_cell(u, N, i, j, k, ih2, bC, q, NULL));
                    if (!(r <= lm)) lm = r; /* NaN propagates */
                }
#pragma omp critical
        mx = nanmax(mx, lm);
    }
    return mx;
}

/* One red-black Newton-Gauss-Seidel sweep (Sec. 3.3, Eq. iterative_correction):
 * first every red cell ((i+j+k) even) is updated from its six neighbours,
 * then every black cell, each by u <- u - (L - f) / (dL/du).  The paper
 * names no safeguard; a step limit |du| <= max_du (off when max_du <= 0) keeps
 * a cold start from overshooting into overflow of e^{-u/(n+1)} in deeply
 * screened cells, where the curvature term makes the update strongly convex. */
void or_ngs_sweep(int N, double h, double bC, int n, double max_du, double *u, const double *f)
{
    double ih2 = 1.0 / (h * h), q = 1.0 / (n + 1);
    for (int colour = 0; colour < 2; ++colour)
        /* the cells of one colour have neighbours of the other colour only */
#pragma omp parallel for
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j)
                for (int k = 0; k < N; ++k) {
                    if (((i + j + k) & 1) != colour) continue;
                    double J;
                    double L = op_cell(u, N, i, j, k, ih2, bC, q, &J);
                    double du = -(L - f[IDX(i, j, k)]) / J;
                    if (max_du > 0.0) du = fmin(fmax(du, -max_du), max_du);
                    u[IDX(i, j, k)] += du;
                }
}

/* ------------------------------------------------------------- grid transfer */

/* Restriction R (Sec. 3.3): a parent value is the mean of its 8 daughters. */
void or_restrict(int Nf, const double *fine, double *coarse)
{
    int N = Nf / 2;
#pragma omp parallel for
    for (int I = 0; I < N; ++I)
        for (int J = 0; J < N; ++J)
            for (int K = 0; K < N; ++K) {
                double s = 0.0;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b)
                        for (int c = 0; c < 2; ++c)
                            s += fine[(((size_t)(2 * I + a)) * Nf + (2 * J + b)) * Nf + (2 * K + c)];
                coarse[IDX(I, J, K)] = s / 8.0;
            }
}

/* Fine-grid correction u += P(uc - ubar) (Sec. 3.3, Eq. fine_correction).
 * P is straight injection (mode 1) or the linear reconstruction from the
 * parent value and the central-difference gradient at the parent centre
 * (mode 0): a daughter displaced by s_d h/2 (s_d = -1 or +1) along axis d
 * gets e_P + sum_d s_d (e_{P+d} - e_{P-d}) / 8.  Periodic. */
void or_prolong_add(int Nf, int mode, const double *uc, const double *ubar, double *u)
{
    int N = Nf / 2;
#pragma omp parallel for
    for (int i = 0; i < Nf; ++i)
        for (int j = 0; j < Nf; ++j)
            for (int k = 0; k < Nf; ++k) {
                int I = i / 2, J = j / 2, K = k / 2;
#define E(a, b, c) (uc[IDX(a, b, c)] - ubar[IDX(a, b, c)])
                double v = E(I, J, K);
                if (mode == 0) {
                    double si = (i & 1) ? 1.0 : -1.0, sj = (j & 1) ? 1.0 : -1.0, sk = (k & 1) ? 1.0 : -1.0;
                    v += si * (E((I + 1) % N, J, K) - E((I + N - 1) % N, J, K)) / 8.0;
                    v += sj * (E(I, (J + 1) % N, K) - E(I, (J + N - 1) % N, K)) / 8.0;
                    v += sk * (E(I, J, (K + 1) % N) - E(I, J, (K + N - 1) % N)) / 8.0;
                }
#undef E
                u[(((size_t)i) * Nf + j) * Nf + k] += v;
            }
}

/* ---------------------------------------------------------------- multigrid */

typedef struct {
    int nlev;
    int Ns[32];
    double hs[32];
    double *u[32], *f[32], *ubar[32], *tmp[32];
} or_hier;

static void hier_free(or_hier *H)
{
    for (int l = 0; l < H->nlev; ++l) {
        if (l > 0) { free(H->u[l]); free(H->f[l]); }
        free(H->ubar[l]);
        free(H->tmp[l]);
    }
}

/* One FAS V-cycle on level l (Sec. 3.3, steps 3-7). */
static void vcycle(or_hier *H, int l, const or_params *p, double bC)
{
    int N = H->Ns[l];
    double h = H->hs[l];
    if (l == H->nlev - 1) { /* coarsest (4^3): NGS directly */
        for (int s = 0; s < p->coarse_sweeps; ++s) or_ngs_sweep(N, h, bC, p->n, p->max_du, H->u[l], H->f[l]);
        return;
    }
    for (int s = 0; s < p->pre_smooth; ++s) or_ngs_sweep(N, h, bC, p->n, p->max_du, H->u[l], H->f[l]);
    size_t n3 = (size_t)N * N * N;
    int Nc = H->Ns[l + 1];
    size_t nc3 = (size_t)Nc * Nc * Nc;
    /* residual r = f - L(u) on this level */
    or_apply_L(N, h, bC, p->n, H->u[l], H->tmp[l]);
#pragma omp parallel for
    for (size_t c = 0; c < n3; ++c) H->tmp[l][c] = H->f[l][c] - H->tmp[l][c];
    /* coarse problem: f_c = L_c(R u) + R(f - L(u)), initial guess R u */
    or_restrict(N, H->u[l], H->ubar[l + 1]);
    or_restrict(N, H->tmp[l], H->f[l + 1]);
    or_apply_L(Nc, H->hs[l + 1], bC, p->n, H->ubar[l + 1], H->tmp[l + 1]);
#pragma omp parallel for
    for (size_t c = 0; c < nc3; ++c) H->f[l + 1][c] += H->tmp[l + 1][c];
    memcpy(H->u[l + 1], H->ubar[l + 1], nc3 * sizeof(double));
    vcycle(H, l + 1, p, bC);
    or_prolong_add(N, p->prolong, H->u[l + 1], H->ubar[l + 1], H->u[l]);
    for (int s = 0; s < p->post_smooth; ++s) or_ngs_sweep(N, h, bC, p->n, p->max_du, H->u[l], H->f[l]);
}

/* Number of levels from N down to the 4^3 coarsest grid (Sec. 3.3, step 5). */
int or_num_levels(int N)
{
    int l = 1;
    while (N > 4) { N /= 2; ++l; }
    return l;
}

/* Solve L(u) = f for u on the periodic N^3 mesh (Sec. 3.3, steps 1-8).
 * u holds the initial guess on entry (0 = background) and the result on exit;
 * dfr (nullable) receives delta f_R = fbar_R (e^u - 1) = -|fbar| expm1(u).
 * Acceptance: max |f - L(u)| / D <= tol with D = max |f| (beta C if f == 0),
 * tested before the first cycle and after every cycle. */
int or_solve(const or_params *p, const double *delta, double *u, double *dfr, or_stats *st)
{
    int N = p->mesh;
    double fb, beta, C;
    or_background(p, &fb, &beta, &C);
    double bC = beta * C;
    or_hier H;
    memset(&H, 0, sizeof H);
    H.nlev = or_num_levels(N);
    for (int l = 0, n = N; l < H.nlev; ++l, n /= 2) {
        size_t n3 = (size_t)n * n * n;
        H.Ns[l] = n;
        H.hs[l] = p->box / n;
        H.u[l] = l ? malloc(n3 * sizeof(double)) : u;
        H.f[l] = l ? malloc(n3 * sizeof(double)) : malloc(n3 * sizeof(double));
        H.ubar[l] = malloc(n3 * sizeof(double));
        H.tmp[l] = malloc(n3 * sizeof(double));
    }
    size_t n3 = (size_t)N * N * N;
    or_source(p, delta, H.f[0]);
    double D = 0.0;
    for (size_t c = 0; c < n3; ++c) if (!(fabs(H.f[0][c]) <= D)) D = fabs(H.f[0][c]);
    if (D == 0.0) D = bC;
    memset(st, 0, sizeof *st);
    st->scale = D;
    int status = 1;
    double res = or_residual_max(N, H.hs[0], bC, p->n, u, H.f[0]) / D;
    st->res0 = res;
    int cyc = 0;
    for (;;) {
        if (!isfinite(res)) { status = -3; break; }
        if (res <= p->tol) { status = 0; break; }
        if (cyc >= p->max_vcycles) { status = 1; break; }
        vcycle(&H, 0, p, bC);
        res = or_residual_max(N, H.hs[0], bC, p->n, u, H.f[0]) / D;
        if (cyc < OR_MAX_HIST) st->res_hist[cyc] = res;
        ++cyc;
    }
    st->vcycles = cyc;
    st->res = res;
    st->status = status;
    if (dfr) {
#pragma omp parallel for
        for (size_t c = 0; c < n3; ++c) dfr[c] = -fb * expm1(u[c]);
    }
    free(H.f[0]);
    hier_free(&H);
    return status;
}

/* One V-cycle on a given level set-up, exposed for per-step parity tests. */
void or_vcycle_once(const or_params *p, const double *f, double *u)
{
    int N = p->mesh;
    double fb, beta, C;
    or_background(p, &fb, &beta, &C);
    or_hier H;
    memset(&H, 0, sizeof H);
    H.nlev = or_num_levels(N);
    for (int l = 0, n = N; l < H.nlev; ++l, n /= 2) {
        size_t n3 = (size_t)n * n * n;
        H.Ns[l] = n;
        H.hs[l] = p->box / n;
        H.u[l] = l ? malloc(n3 * sizeof(double)) : u;
        H.f[l] = l ? malloc(n3 * sizeof(double)) : malloc(n3 * sizeof(double));
        H.ubar[l] = malloc(n3 * sizeof(double));
        H.tmp[l] = malloc(n3 * sizeof(double));
    }
    memcpy(H.f[0], f, sizeof(double) * (size_t)N * N * N);
    vcycle(&H, 0, p, beta * C);
    free(H.f[0]);
    hier_free(&H);
}

/* ------------------------------------------------------------- fifth force */

/* a_MG = (c^2/2) grad_phys f_R (Sec. 2, Eq. modgrav_accel) = c^2/(2a) grad_x f_R
 * in comoving x, f_R = fbar_R e^u.  The gradient at cell centres is the
 * two-point central difference; it is interpolated to the particles with
 * the same cloud-in-cell weights as the mass assignment.  Units of acc:
 * (km/s)^2 h/Mpc. */
void or_fifth_force(const or_params *p, const double *u, int64_t np, const float *pos, double *acc)
{
    int N = p->mesh;
    double h = p->box / N;
    double fb, beta, C;
    or_background(p, &fb, &beta, &C);
    size_t n3 = (size_t)N * N * N;
    double *fr = malloc(n3 * sizeof(double));
    double *g = malloc(3 * n3 * sizeof(double));
#pragma omp parallel for
    for (size_t c = 0; c < n3; ++c) fr[c] = -fb * exp(u[c]);
#pragma omp parallel for
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
            for (int k = 0; k < N; ++k) {
                size_t c = IDX(i, j, k);
                g[3 * c + 0] = (fr[IDX((i + 1) % N, j, k)] - fr[IDX((i + N - 1) % N, j, k)]) / (2 * h);
                g[3 * c + 1] = (fr[IDX(i, (j + 1) % N, k)] - fr[IDX(i, (j + N - 1) % N, k)]) / (2 * h);
                g[3 * c + 2] = (fr[IDX(i, j, (k + 1) % N)] - fr[IDX(i, j, (k + N - 1) % N)]) / (2 * h);
            }
    double pref = OR_C_KMS * OR_C_KMS / (2.0 * p->a);
#pragma omp parallel for
    for (int64_t q = 0; q < np; ++q) {
        long i0[3];
        double t[3];
        for (int d = 0; d < 3; ++d) {
            double xi = (double)pos[3 * q + d] / h - 0.5;
            double fl = floor(xi);
            t[d] = xi - fl;
            i0[d] = (long)fl;
        }
        double s[3] = {0, 0, 0};
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int c = 0; c < 2; ++c) {
                    double w = (a ? t[0] : 1.0 - t[0]) * (b ? t[1] : 1.0 - t[1]) *
                               (c ? t[2] : 1.0 - t[2]);
                    size_t cell = ((size_t)wrapi(i0[0] + a, N) * N + wrapi(i0[1] + b, N)) * N +
                                  wrapi(i0[2] + c, N);
                    for (int d = 0; d < 3; ++d) s[d] += w * g[3 * cell + d];
                }
        for (int d = 0; d < 3; ++d) acc[3 * q + d] = pref * s[d];
    }
    free(fr);
    free(g);
}

/* ------------------------------------------------- sampled checks (large meshes) */

/* Residual f - L(u) at `count` listed cells (flat C-order indices). */
void or_residual_at(int N, double h, double bC, int n, const double *u, const double *f, int64_t count,
                    const int64_t *cells, double *out)
{
    double ih2 = 1.0 / (h * h), q = 1.0 / (n + 1);
#pragma omp parallel for
    for (int64_t s = 0; s < count; ++s) {
        int64_t c = cells[s];
        int k = (int)(c % N), j = (int)((c / N) % N), i = (int)(c / ((int64_t)N * N));
        out[s] = f[c] - op_cell(u, N, i, j, k, ih2, bC, q, NULL);
    }
}

/* Cloud-in-cell mass of `count` listed cells, scanning every particle
 * (same weights as or_cic_assign; `mark` is caller scratch of N^3 bytes). */
void or_cic_cells(int N, double box, int64_t np, const float *pos, const double *mass, int64_t count,
                  const int64_t *cells, unsigned char *mark, double *out)
{
    double h = box / N;
    size_t n3 = (size_t)N * N * N;
    memset(mark, 0, n3);
    for (int64_t s = 0; s < count; ++s) { mark[cells[s]] = 1; out[s] = 0.0; }
    for (int64_t p = 0; p < np; ++p) {
        long i0[3];
        double t[3];
        for (int d = 0; d < 3; ++d) {
            double xi = (double)pos[3 * p + d] / h - 0.5;
            double fl = floor(xi);
            t[d] = xi - fl;
            i0[d] = (long)fl;
        }
        double mp = mass ? mass[p] : 1.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int c = 0; c < 2; ++c) {
                    size_t cell = ((size_t)wrapi(i0[0] + a, N) * N + wrapi(i0[1] + b, N)) * N + wrapi(i0[2] + c, N);
                    if (!mark[cell]) continue;
                    double w = (a ? t[0] : 1.0 - t[0]) * (b ? t[1] : 1.0 - t[1]) * (c ? t[2] : 1.0 - t[2]);
                    for (int64_t s = 0; s < count; ++s)
                        if ((size_t)cells[s] == cell) out[s] += w * mp;
                }
    }
}

/* Fifth force (as or_fifth_force) at `np` particles, f_R evaluated on the fly. */
void or_fifth_force_at(const or_params *p, const double *u, int64_t np, const float *pos, double *acc)
{
    int N = p->mesh;
    double h = p->box / N;
    double fb, beta, C;
    or_background(p, &fb, &beta, &C);
    double pref = OR_C_KMS * OR_C_KMS / (2.0 * p->a);
#define FR(i, j, k) (-fb * exp(u[((size_t)wrapi(i, N) * N + wrapi(j, N)) * N + wrapi(k, N)]))
#pragma omp parallel for
    for (int64_t q = 0; q < np; ++q) {
        long i0[3];
        double t[3];
        for (int d = 0; d < 3; ++d) {
            double xi = (double)pos[3 * q + d] / h - 0.5;
            double fl = floor(xi);
            t[d] = xi - fl;
            i0[d] = (long)fl;
        }
        double s[3] = {0, 0, 0};
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int c = 0; c < 2; ++c) {
                    double w = (a ? t[0] : 1.0 - t[0]) * (b ? t[1] : 1.0 - t[1]) * (c ? t[2] : 1.0 - t[2]);
                    long i = i0[0] + a, j = i0[1] + b, k = i0[2] + c;
                    s[0] += w * (FR(i + 1, j, k) - FR(i - 1, j, k)) / (2 * h);
                    s[1] += w * (FR(i, j + 1, k) - FR(i, j - 1, k)) / (2 * h);
                    s[2] += w * (FR(i, j, k + 1) - FR(i, j, k - 1)) / (2 * h);
                }
        for (int d = 0; d < 3; ++d) acc[3 * q + d] = pref * s[d];
    }
#undef FR
}

/* ------------------------------------------------------------- refined levels
 *
 * Block-structured adaptive refinement with the paper's one-way interface
 * (Sec. 3.3, steps 9-12).  Level l has N_l = N_0 2^l cells per side.  A cell
 * of level l-1 holding more than 8 particles (nearest-grid-point count) is
 * refined: its children and those of the aligned 4^3 group of level-(l-1)
 * cells around it form an 8^3 block of level l.  Level-2 blocks also refine
 * every level-1 block within two level-1 cells of them, so that the ghost
 * cells of level 2 and the parents they are prolonged from lie on level 1.
 * Each level is solved after its parent: the initial guess and the ghost layer
 * around the union of blocks come from the linear prolongation of the parent
 * solution (fixed during the level solve), and the level is solved by FAS
 * V-cycles whose coarse grids are the union of blocks at 1/2, 1/4 and 1/8
 * resolution (one cell per block at the coarsest; every coarse cell is fully
 * covered, so the paper's mask is 1 on all of them); coarse cells outside the
 * union hold the parent solution at that resolution (restricted from the base
 * below the base resolution) and are never updated.
 *
 * Dense storage: every level is an N_l^3 array with a mask; this oracle only
 * needs small meshes.                                                         */

#define OR_AMR_MAXL 3

typedef struct {
    int N;            /* side at this resolution */
    double h;
    unsigned char *mask; /* 1 = unknown of the level solve */
    double *u, *f, *fr;  /* fr: frozen values outside the mask */
    double *ubar, *r;
} or_sub;

static size_t cube(int n) { return (size_t)n * n * n; }

#define SIDX(S, i, j, k) ((((size_t)wrapi(i, (S)->N)) * (S)->N + wrapi(j, (S)->N)) * (S)->N + wrapi(k, (S)->N))

static double sval(const or_sub *S, long i, long j, long k)
{
    size_t c = SIDX(S, i, j, k);
    return S->mask[c] ? S->u[c] : S->fr[c];
}

/* L and dL/du at a masked cell, neighbours from the unknowns or the frozen values */
static double sub_op(const or_sub *S, int i, int j, int k, double bC, double q, double *J)
{
    double ih2 = 1.0 / (S->h * S->h);
    double uc = S->u[SIDX(S, i, j, k)];
    double nb[6] = {sval(S, i + 1, j, k), sval(S, i - 1, j, k), sval(S, i, j + 1, k),
                    sval(S, i, j - 1, k), sval(S, i, j, k + 1), sval(S, i, j, k - 1)};
    double ec = exp(uc), lap = 0.0, dlap = 0.0;
    for (int s = 0; s < 6; ++s) {
        double en = exp(nb[s]);
        lap += 0.5 * (en + ec) * (nb[s] - uc);
        dlap += 0.5 * (ec * (nb[s] - uc - 1.0) - en);
    }
    double em = expm1(-q * uc);
    if (J) *J = ih2 * dlap - bC * q * (1.0 + em);
    return ih2 * lap + bC * em;
}

static void sub_sweep(or_sub *S, double bC, double q, double max_du)
{
    int N = S->N;
    for (int colour = 0; colour < 2; ++colour)
#pragma omp parallel for
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j)
                for (int k = 0; k < N; ++k) {
                    size_t c = ((size_t)i * N + j) * N + k;
                    if (!S->mask[c] || ((i + j + k) & 1) != colour) continue;
                    double J;
                    double L = sub_op(S, i, j, k, bC, q, &J);
                    double du = -(L - S->f[c]) / J;
                    if (max_du > 0.0) du = fmin(fmax(du, -max_du), max_du);
                    S->u[c] += du;
                }
}

static double sub_resmax(or_sub *S, double bC, double q)
{
    int N = S->N;
    double mx = 0.0;
#pragma omp parallel
    {
        double lm = 0.0;
#pragma omp for
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j)
                for (int k = 0; k < N; ++k) {
                    size_t c = ((size_t)i * N + j) * N + k;
                    if (!S->mask[c]) continue;
                    double r = fabs(S->f[c] - sub_op(S, i, j, k, bC, q, NULL));
                    if (!(r <= lm)) lm = r;
                }
#pragma omp critical
        mx = nanmax(mx, lm);
    }
    return mx;
}

static void amr_vcycle(or_sub *Sv, int m, int nsub, const or_params *p, double bC, double q)
{
    or_sub *S = &Sv[m];
    if (m == nsub - 1) {
        for (int s = 0; s < p->coarse_sweeps; ++s) sub_sweep(S, bC, q, p->max_du);
        return;
    }
    for (int s = 0; s < p->pre_smooth; ++s) sub_sweep(S, bC, q, p->max_du);
    int N = S->N;
#pragma omp parallel for
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
            for (int k = 0; k < N; ++k) {
                size_t c = ((size_t)i * N + j) * N + k;
                S->r[c] = S->mask[c] ? S->f[c] - sub_op(S, i, j, k, bC, q, NULL) : 0.0;
            }
    or_sub *C = &Sv[m + 1];
    int Nc = C->N;
    for (int I = 0; I < Nc; ++I)
        for (int Jx = 0; Jx < Nc; ++Jx)
            for (int K = 0; K < Nc; ++K) {
                size_t cc = ((size_t)I * Nc + Jx) * Nc + K;
                if (!C->mask[cc]) continue;
                double su = 0.0, sr = 0.0;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b)
                        for (int d = 0; d < 2; ++d) {
                            size_t fc = (((size_t)(2 * I + a)) * N + (2 * Jx + b)) * N + (2 * K + d);
                            su += S->u[fc];
                            sr += S->r[fc];
                        }
                C->ubar[cc] = su / 8.0;
                C->f[cc] = sr / 8.0;
            }
    for (size_t cc = 0; cc < cube(Nc); ++cc) if (C->mask[cc]) C->u[cc] = C->ubar[cc];
    for (int I = 0; I < Nc; ++I)
        for (int Jx = 0; Jx < Nc; ++Jx)
            for (int K = 0; K < Nc; ++K) {
                size_t cc = ((size_t)I * Nc + Jx) * Nc + K;
                if (C->mask[cc]) C->f[cc] += sub_op(C, I, Jx, K, bC, q, NULL);
            }
    amr_vcycle(Sv, m + 1, nsub, p, bC, q);
    /* correction u += P(e), e = u_c - ubar on the coarse unknowns and 0 elsewhere */
#define EC(a, b, c) (C->mask[SIDX(C, a, b, c)] ? C->u[SIDX(C, a, b, c)] - C->ubar[SIDX(C, a, b, c)] : 0.0)
#pragma omp parallel for
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
            for (int k = 0; k < N; ++k) {
                size_t c = ((size_t)i * N + j) * N + k;
                if (!S->mask[c]) continue;
                int I = i / 2, Jx = j / 2, K = k / 2;
                double v = EC(I, Jx, K);
                if (p->prolong == 0) {
                    double si = (i & 1) ? 1.0 : -1.0, sj = (j & 1) ? 1.0 : -1.0, sk = (k & 1) ? 1.0 : -1.0;
                    v += si * (EC(I + 1, Jx, K) - EC(I - 1, Jx, K)) / 8.0;
                    v += sj * (EC(I, Jx + 1, K) - EC(I, Jx - 1, K)) / 8.0;
                    v += sk * (EC(I, Jx, K + 1) - EC(I, Jx, K - 1)) / 8.0;
                }
                S->u[c] += v;
            }
#undef EC
    for (int s = 0; s < p->post_smooth; ++s) sub_sweep(S, bC, q, p->max_du);
}

/* linear prolongation of a full field (values, not corrections) to cell (i,j,k) of a
 * mesh of side 2N from the side-N field P (periodic) */
static double prolong_field_at(const double *P, int N, long i, long j, long k)
{
    long I = i / 2, J = j / 2, K = k / 2;
    if (i < 0) I = (i - 1) / 2;
    if (j < 0) J = (j - 1) / 2;
    if (k < 0) K = (k - 1) / 2;
#define PV(a, b, c) P[((size_t)wrapi(a, N) * N + wrapi(b, N)) * N + wrapi(c, N)]
    double v = PV(I, J, K);
    double si = (wrapi(i, 2 * N) & 1) ? 1.0 : -1.0, sj = (wrapi(j, 2 * N) & 1) ? 1.0 : -1.0,
           sk = (wrapi(k, 2 * N) & 1) ? 1.0 : -1.0;
    v += si * (PV(I + 1, J, K) - PV(I - 1, J, K)) / 8.0;
    v += sj * (PV(I, J + 1, K) - PV(I, J - 1, K)) / 8.0;
    v += sk * (PV(I, J, K + 1) - PV(I, J, K - 1)) / 8.0;
#undef PV
    return v;
}

/* Block index of cell (i,j,k) (any integers, wrapped) of a level with N cells
 * per side, in its map of (N/8)^3 block positions. */
static size_t blk_of(int N, long i, long j, long k)
{
    int M = N / 8;
    return ((size_t)(wrapi(i, N) / 8) * M + wrapi(j, N) / 8) * M + wrapi(k, N) / 8;
}

/* Refinement flags (reading of Sec. 3.1's rule that an AMR cell holds at most
 * eight particles, for 8^3-cell blocks).  blk[l] (l = 1..nref) are caller
 * arrays of (N_l/8)^3 bytes, N_l = N_0 2^l, set to 1 where level l has a
 * block.  A cell of level l-1 holding more than 8 particles (nearest-grid-
 * point count) refines the aligned 4^3 group of level-(l-1) cells around it;
 * on level 1 only particles inside level-1 blocks count.  Proper nesting: every
 * level-1 block with a level-1 cell within two cells of a level-2 block is
 * refined too, so that the ghost cells of level 2 and the parents they are
 * prolonged from lie on level 1. */
void or_amr_flags(const or_params *p, int nref, int64_t np, const float *pos, unsigned char **blk)
{
    int N0 = p->mesh;
    for (int l = 1; l <= nref; ++l) memset(blk[l], 0, cube((N0 << l) / 8));
    if (nref <= 0) return;
    {   /* level 1 from base counts */
        int *cnt = calloc(cube(N0), sizeof(int));
        double h = p->box / N0;
        for (int64_t i = 0; i < np; ++i) {
            long c[3];
            for (int d = 0; d < 3; ++d) c[d] = wrapi((long)floor((double)pos[3 * i + d] / h), N0);
            cnt[((size_t)c[0] * N0 + c[1]) * N0 + c[2]]++;
        }
        int nb = N0 / 4;
        for (int i = 0; i < N0; ++i)
            for (int j = 0; j < N0; ++j)
                for (int k = 0; k < N0; ++k)
                    if (cnt[((size_t)i * N0 + j) * N0 + k] > 8) blk[1][((size_t)(i / 4) * nb + j / 4) * nb + k / 4] = 1;
        free(cnt);
    }
    if (nref >= 2) {  /* level 2 from level-1 counts inside level-1 blocks */
        int N1 = 2 * N0, nb2 = N1 / 4;
        int *cnt = calloc(cube(N1), sizeof(int));
        double h = p->box / N1;
        for (int64_t i = 0; i < np; ++i) {
            long c[3];
            for (int d = 0; d < 3; ++d) c[d] = wrapi((long)floor((double)pos[3 * i + d] / h), N1);
            if (blk[1][blk_of(N1, c[0], c[1], c[2])]) cnt[((size_t)c[0] * N1 + c[1]) * N1 + c[2]]++;
        }
        for (int i = 0; i < N1; ++i)
            for (int j = 0; j < N1; ++j)
                for (int k = 0; k < N1; ++k)
                    if (cnt[((size_t)i * N1 + j) * N1 + k] > 8) blk[2][((size_t)(i / 4) * nb2 + j / 4) * nb2 + k / 4] = 1;
        free(cnt);
        /* proper nesting: level-1 blocks within two level-1 cells of every level-2 block */
        for (int bi = 0; bi < nb2; ++bi)
            for (int bj = 0; bj < nb2; ++bj)
                for (int bk = 0; bk < nb2; ++bk) {
                    if (!blk[2][((size_t)bi * nb2 + bj) * nb2 + bk]) continue;
                    for (long ci = 4L * bi - 2; ci < 4L * bi + 6; ++ci)
                        for (long cj = 4L * bj - 2; cj < 4L * bj + 6; ++cj)
                            for (long ck = 4L * bk - 2; ck < 4L * bk + 6; ++ck) blk[1][blk_of(N1, ci, cj, ck)] = 1;
                }
    }
}

/* Does cell (i,j,k) of level l belong to the composite (leaf) mesh: it lies in
 * a level-l block (every cell of level 0) and no level-(l+1) block covers it. */
static int amr_leaf(int N0, int nref, unsigned char **blk, int l, long i, long j, long k)
{
    int N = N0 << l;
    if (l >= 1 && !blk[l][blk_of(N, i, j, k)]) return 0;
    /* the children of (i,j,k) are level-(l+1) cells 2i.., in block 2i/8 = i/4 */
    if (l < nref && blk[l + 1][blk_of(2 * N, 2 * wrapi(i, N), 2 * wrapi(j, N), 2 * wrapi(k, N))]) return 0;
    return 1;
}

/* Cloud-in-cell masses on the composite mesh (Sec. 3.1): a particle is a cube
 * whose side is that of the finest cell containing it, and every leaf cell
 * that the cube overlaps -- of whatever level -- receives the particle's mass
 * times the overlapping fraction of the cube's volume; then each coarser
 * cell covered by a finer level gets the sum of its eight daughters' masses.
 * m[l]: caller arrays of N_l^3 doubles (cells outside level l's blocks end at
 * 0).  mass == NULL means unit masses.  With nref = 0 this is or_cic_assign. */
void or_amr_cic(const or_params *p, int nref, unsigned char **blk, int64_t np, const float *pos,
                const double *mass, double **m)
{
    int N0 = p->mesh;
    for (int l = 0; l <= nref; ++l) memset(m[l], 0, cube(N0 << l) * sizeof(double));
    for (int64_t q = 0; q < np; ++q) {
        double x[3];
        for (int d = 0; d < 3; ++d) x[d] = (double)pos[3 * q + d];
        int lp = 0; /* finest level whose blocks contain the particle */
        for (int l = nref; l >= 1 && !lp; --l) {
            double hl = p->box / (N0 << l);
            if (blk[l][blk_of(N0 << l, (long)floor(x[0] / hl), (long)floor(x[1] / hl), (long)floor(x[2] / hl))]) lp = l;
        }
        double s = p->box / (N0 << lp), mp = mass ? mass[q] : 1.0;
        double lo[3], hi[3];
        for (int d = 0; d < 3; ++d) { lo[d] = x[d] - 0.5 * s; hi[d] = x[d] + 0.5 * s; }
        for (int l = 0; l <= nref; ++l) {
            int N = N0 << l;
            double h = p->box / N;
            long c0[3], c1[3];
            for (int d = 0; d < 3; ++d) { c0[d] = (long)floor(lo[d] / h); c1[d] = (long)floor(hi[d] / h); }
            for (long i = c0[0]; i <= c1[0]; ++i)
                for (long j = c0[1]; j <= c1[1]; ++j)
                    for (long k = c0[2]; k <= c1[2]; ++k) {
                        long c[3] = {i, j, k};
                        double v = 1.0;
                        for (int d = 0; d < 3; ++d) {
                            double a = fmax(lo[d], c[d] * h), b = fmin(hi[d], (c[d] + 1) * h);
                            v *= b > a ? (b - a) / s : 0.0;
                        }
                        if (v <= 0.0 || !amr_leaf(N0, nref, blk, l, i, j, k)) continue;
                        m[l][((size_t)wrapi(i, N) * N + wrapi(j, N)) * N + wrapi(k, N)] += mp * v;
                    }
        }
    }
    /* coarser cells covered by a finer level: the sum of their daughters */
    for (int l = nref - 1; l >= 0; --l) {
        int N = N0 << l, Nf = 2 * N;
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j)
                for (int k = 0; k < N; ++k) {
                    if (!blk[l + 1][blk_of(Nf, 2 * i, 2 * j, 2 * k)]) continue;
                    double sum = 0.0;
                    for (int a = 0; a < 2; ++a)
                        for (int b = 0; b < 2; ++b)
                            for (int c = 0; c < 2; ++c)
                                sum += m[l + 1][((size_t)(2 * i + a) * Nf + (2 * j + b)) * Nf + (2 * k + c)];
                    m[l][((size_t)i * N + j) * N + k] = sum;
                }
    }
}

/* Solve the base mesh and `nref` (0..2) refined levels (Sec. 3.3, steps 1-12)
 * for given density contrasts.  blk[l]: the levels' block maps (as from
 * or_amr_flags; proper nesting is the caller's business); delta[l]: N_l^3
 * arrays, used on level l's block cells (delta[0] everywhere).  u[l], mask[l]:
 * caller arrays of N_l^3 elements; u[l] receives the level-l solution on its
 * block cells (u[0] everywhere, solved from u = 0), mask[l] the block cells.
 * st[l]: per-level statistics.  Returns the worst status. */
int or_amr_solve_fields(const or_params *p, int nref, unsigned char **blk, double **delta, double **u,
                        unsigned char **mask, or_stats *st)
{
    int N0 = p->mesh;
    double fb, beta, C;
    or_background(p, &fb, &beta, &C);
    double bC = beta * C, q = 1.0 / (p->n + 1);
    double srcs = beta * p->omega_m / (p->a * p->a * p->a);
    memset(u[0], 0, cube(N0) * sizeof(double));
    int worst = or_solve(p, delta[0], u[0], NULL, &st[0]);
    memset(mask[0], 1, cube(N0));
    for (int l = 1; l <= nref; ++l) {
        int N = N0 << l;
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j)
                for (int k = 0; k < N; ++k) mask[l][((size_t)i * N + j) * N + k] = blk[l][blk_of(N, i, j, k)];
    }
    /* level solves, coarse to fine */
    for (int l = 1; l <= nref; ++l) {
        int N = N0 << l;
        or_sub Sv[4];
        int nsub = 4;
        for (int m = 0; m < nsub; ++m) {
            int Nm = N >> m;
            or_sub *S = &Sv[m];
            S->N = Nm;
            S->h = p->box / Nm;
            S->mask = calloc(cube(Nm), 1);
            S->u = calloc(cube(Nm), sizeof(double));
            S->f = calloc(cube(Nm), sizeof(double));
            S->fr = calloc(cube(Nm), sizeof(double));
            S->ubar = calloc(cube(Nm), sizeof(double));
            S->r = calloc(cube(Nm), sizeof(double));
            for (int i = 0; i < Nm; ++i)
                for (int j = 0; j < Nm; ++j)
                    for (int k = 0; k < Nm; ++k)
                        S->mask[((size_t)i * Nm + j) * Nm + k] =
                            mask[l][(((size_t)(i << m)) * N + (j << m)) * N + (k << m)];
            /* frozen values: the solution at resolution level l - m */
            int lp = l - m;
            for (int i = 0; i < Nm; ++i)
                for (int j = 0; j < Nm; ++j)
                    for (int k = 0; k < Nm; ++k) {
                        size_t c = ((size_t)i * Nm + j) * Nm + k;
                        double v;
                        if (m == 0) {
                            v = prolong_field_at(u[l - 1], N / 2, i, j, k);
                        } else if (lp >= 1) {
                            v = u[lp][c];
                        } else if (lp == 0) {
                            v = u[0][c];
                        } else {
                            int f = 1 << (-lp);
                            double s = 0.0;
                            for (int a = 0; a < f; ++a)
                                for (int b = 0; b < f; ++b)
                                    for (int d = 0; d < f; ++d)
                                        s += u[0][(((size_t)(i * f + a)) * N0 + (j * f + b)) * N0 + (k * f + d)];
                            v = s / (f * f * f);
                        }
                        S->fr[c] = v;
                    }
        }
        /* unknowns, source and initial guess on level l */
        or_sub *S0 = &Sv[0];
        double D = 0.0;
        for (size_t c = 0; c < cube(N); ++c) {
            if (!S0->mask[c]) continue;
            S0->f[c] = srcs * delta[l][c];
            S0->u[c] = S0->fr[c];
            if (fabs(S0->f[c]) > D) D = fabs(S0->f[c]);
        }
        if (D == 0.0) D = bC;
        or_stats *s = &st[l];
        memset(s, 0, sizeof *s);
        s->scale = D;
        double res = sub_resmax(S0, bC, q) / D;
        s->res0 = res;
        int cyc = 0, status;
        for (;;) {
            if (!isfinite(res)) { status = -3; break; }
            if (res <= p->tol) { status = 0; break; }
            if (cyc >= p->max_vcycles) { status = 1; break; }
            amr_vcycle(Sv, 0, nsub, p, bC, q);
            res = sub_resmax(S0, bC, q) / D;
            if (cyc < OR_MAX_HIST) s->res_hist[cyc] = res;
            ++cyc;
        }
        s->vcycles = cyc;
        s->res = res;
        s->status = status;
        if (status != 0 && (worst == 0 || status < 0)) worst = status;
        for (size_t c = 0; c < cube(N); ++c) u[l][c] = S0->mask[c] ? S0->u[c] : 0.0;
        for (int m = 0; m < nsub; ++m) {
            free(Sv[m].mask); free(Sv[m].u); free(Sv[m].f); free(Sv[m].fr); free(Sv[m].ubar); free(Sv[m].r);
        }
    }
    return worst;
}

/* The adaptive solve for np unit-mass particles: refinement flags
 * (or_amr_flags), composite cloud-in-cell masses (or_amr_cic), delta_l =
 * m_l / mbar_l - 1 with mbar_l the total mass over N_l^3 (the mean cell mass
 * at level l's resolution, so a parent's delta is the mean of its
 * daughters'), then or_amr_solve_fields. */
int or_amr_solve(const or_params *p, int nref, int64_t np, const float *pos, double **u, unsigned char **mask,
                 or_stats *st)
{
    int N0 = p->mesh;
    unsigned char *blk[OR_AMR_MAXL] = {0};
    double *m[OR_AMR_MAXL] = {0};
    for (int l = 1; l <= nref; ++l) blk[l] = calloc(cube((N0 << l) / 8), 1);
    for (int l = 0; l <= nref; ++l) m[l] = malloc(cube(N0 << l) * sizeof(double));
    or_amr_flags(p, nref, np, pos, blk);
    or_amr_cic(p, nref, blk, np, pos, NULL, m);
    double total = 0.0;
    for (size_t c = 0; c < cube(N0); ++c) total += m[0][c];
    for (int l = 0; l <= nref; ++l) {
        double mbar = total / (double)cube(N0 << l);
        for (size_t c = 0; c < cube(N0 << l); ++c) m[l][c] = m[l][c] / mbar - 1.0;
    }
    int worst = or_amr_solve_fields(p, nref, blk, m, u, mask, st);
    for (int l = 0; l <= nref; ++l) free(m[l]);
    for (int l = 1; l <= nref; ++l) free(blk[l]);
    return worst;
}

/* ------------------------------------------------ sampled checks of the adaptive mesh */

static int key_cmp(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : x > y;
}

static uint64_t cell_key(int l, long i, long j, long k)
{
    return ((uint64_t)l << 60) | ((uint64_t)i << 40) | ((uint64_t)j << 20) | (uint64_t)k;
}

/* Composite cloud-in-cell mass (as or_amr_cic) of `count` listed cells, from
 * the np given particles: lev[s] is the level of cell s and ijk[3s..3s+2] its
 * indices there (0 <= index < N_lev < 2^20).  A listed cell that a finer
 * level covers gets the sum over its descendants, as the daughter sums of
 * or_amr_cic give.  mass == NULL means unit masses. */
void or_amr_cic_cells(const or_params *p, int nref, unsigned char **blk, int64_t np, const float *pos,
                      const double *mass, int64_t count, const int *lev, const int *ijk, double *out)
{
    int N0 = p->mesh;
    uint64_t *keys = malloc((size_t)count * sizeof(uint64_t));
    for (int64_t s = 0; s < count; ++s) {
        keys[s] = cell_key(lev[s], ijk[3 * s], ijk[3 * s + 1], ijk[3 * s + 2]);
        out[s] = 0.0;
    }
    uint64_t *sorted = malloc((size_t)count * sizeof(uint64_t));
    memcpy(sorted, keys, (size_t)count * sizeof(uint64_t));
    qsort(sorted, (size_t)count, sizeof(uint64_t), key_cmp);
    for (int64_t q = 0; q < np; ++q) {
        double x[3];
        for (int d = 0; d < 3; ++d) x[d] = (double)pos[3 * q + d];
        int lp = 0;
        for (int l = nref; l >= 1 && !lp; --l) {
            double hl = p->box / (N0 << l);
            if (blk[l][blk_of(N0 << l, (long)floor(x[0] / hl), (long)floor(x[1] / hl), (long)floor(x[2] / hl))]) lp = l;
        }
        double s = p->box / (N0 << lp), mp = mass ? mass[q] : 1.0;
        double lo[3], hi[3];
        for (int d = 0; d < 3; ++d) { lo[d] = x[d] - 0.5 * s; hi[d] = x[d] + 0.5 * s; }
        for (int m = 0; m <= nref; ++m) {
            int N = N0 << m;
            double h = p->box / N;
            long c0[3], c1[3];
            for (int d = 0; d < 3; ++d) { c0[d] = (long)floor(lo[d] / h); c1[d] = (long)floor(hi[d] / h); }
            for (long i = c0[0]; i <= c1[0]; ++i)
                for (long j = c0[1]; j <= c1[1]; ++j)
                    for (long k = c0[2]; k <= c1[2]; ++k) {
                        long c[3] = {i, j, k};
                        double v = 1.0;
                        for (int d = 0; d < 3; ++d) {
                            double a = fmax(lo[d], c[d] * h), b = fmin(hi[d], (c[d] + 1) * h);
                            v *= b > a ? (b - a) / s : 0.0;
                        }
                        if (v <= 0.0 || !amr_leaf(N0, nref, blk, m, i, j, k)) continue;
                        long wi = wrapi(i, N), wj = wrapi(j, N), wk = wrapi(k, N);
                        for (int l = 0; l <= m; ++l) { /* the leaf and each of its ancestors */
                            uint64_t key = cell_key(l, wi >> (m - l), wj >> (m - l), wk >> (m - l));
                            uint64_t *hit = bsearch(&key, sorted, (size_t)count, sizeof(uint64_t), key_cmp);
                            if (!hit) continue;
                            for (int64_t t = 0; t < count; ++t)
                                if (keys[t] == key) out[t] += mp * v;
                        }
                    }
        }
    }
    free(keys);
    free(sorted);
}

/* L_c at `count` cells from explicit stencils: uc[s] and its six neighbours
 * nb[6s..6s+5] in the order +x, -x, +y, -y, +z, -z, on a level of cell side h
 * (the operator of or_apply_L, through op_cell on a 3^3 patch). */
void or_op_stencil(double h, double bC, int n, int64_t count, const double *uc, const double *nb, double *L)
{
    double ih2 = 1.0 / (h * h), q = 1.0 / (n + 1);
    for (int64_t s = 0; s < count; ++s) {
        double u[27];
        for (int c = 0; c < 27; ++c) u[c] = 0.0;
        u[13] = uc[s];
        u[22] = nb[6 * s + 0]; /* (2,1,1) */
        u[4] = nb[6 * s + 1];  /* (0,1,1) */
        u[16] = nb[6 * s + 2]; /* (1,2,1) */
        u[10] = nb[6 * s + 3]; /* (1,0,1) */
        u[14] = nb[6 * s + 4]; /* (1,1,2) */
        u[12] = nb[6 * s + 5]; /* (1,1,0) */
        L[s] = op_cell(u, 3, 1, 1, 1, ih2, bC, q, NULL);
    }
}

/* ---------------------------------------------------- chained particle-mesh steps */

/* pref times the cloud-in-cell interpolation, to each particle, of the
 * two-point central-difference gradient of a cell-centred field (the
 * gradient and weights of or_fifth_force).  acc: [np][3]. */
void or_gather_gradient(int N, double box, const double *field, int64_t np, const float *pos, double pref,
                        double *acc)
{
    double h = box / N;
#pragma omp parallel for
    for (int64_t q = 0; q < np; ++q) {
        long i0[3];
        double t[3];
        for (int d = 0; d < 3; ++d) {
            double xi = (double)pos[3 * q + d] / h - 0.5;
            double fl = floor(xi);
            t[d] = xi - fl;
            i0[d] = (long)fl;
        }
        double s[3] = {0, 0, 0};
#define F(i, j, k) field[((size_t)wrapi(i, N) * N + wrapi(j, N)) * N + wrapi(k, N)]
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int c = 0; c < 2; ++c) {
                    double w = (a ? t[0] : 1.0 - t[0]) * (b ? t[1] : 1.0 - t[1]) * (c ? t[2] : 1.0 - t[2]);
                    long i = i0[0] + a, j = i0[1] + b, k = i0[2] + c;
                    s[0] += w * (F(i + 1, j, k) - F(i - 1, j, k)) / (2 * h);
                    s[1] += w * (F(i, j + 1, k) - F(i, j - 1, k)) / (2 * h);
                    s[2] += w * (F(i, j, k + 1) - F(i, j, k - 1)) / (2 * h);
                }
#undef F
        for (int d = 0; d < 3; ++d) acc[3 * q + d] = pref * s[d];
    }
}

/* Leapfrog kick and drift on float32 particle arrays: mom += acc kick, then
 * pos += mom drift, each in float64 as one fused multiply-add from the float32
 * values and rounded to float32; positions wrapped into [0, box).  acc may be
 * NULL (drift only). */
void or_kick_drift(int64_t np, float *pos, float *mom, const float *acc, double kick, double drift, double box)
{
    for (int64_t t = 0; t < 3 * np; ++t) {
        double m = (double)mom[t];
        if (acc) m = fma((double)acc[t], kick, m);
        mom[t] = (float)m;
        double x = fma((double)mom[t], drift, (double)pos[t]);
        x -= box * floor(x / box);
        pos[t] = (float)x;
    }
}
