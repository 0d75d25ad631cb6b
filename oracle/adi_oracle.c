/*
 * adi_oracle.c -- plain FP64 CPU oracle for the ADI solution of the implicit
 * three-level finite-difference scheme for the 2-D acoustic wave equation
 * (Altybay, Ruzhansky, Tokmagambetov, "A parallel hybrid implementation of the
 * 2D acoustic wave equation", Sec. 2).
 *
 * TEST INFRASTRUCTURE ONLY.  It is called by the test suite, by the smoke
 * check and by the benchmark's CPU-baseline leg; the product library never
 * links, loads or calls it, and it shares no code with the GPU path.
 *
 * What is computed (all in double precision, row-major u[j*nx + i], interior
 * nodes only, the walls being the zero Dirichlet data of eq. (CN3)):
 *
 *   Scheme, eq. (CN1) with a time-independent coefficient kappa(x, y) (the
 *   paper's c, which multiplies the Laplacian in eq. (f1)) and weights 1/2 on
 *   levels k+1 and k-1.  Writing D2 = u^{n+1} - 2u^n + u^{n-1} and
 *   beta = dt^2/2, eq. (CN1) is  (I - beta K Lap) D2 = dt^2 (K Lap u^n + f^n).
 *   The ADI method of Sec. 2 (eqs. (fr1)-(fr2): an x-implicit sub-step, then a
 *   y-implicit sub-step, in that order, see also Sec. 4) replaces the left
 *   operator by the product (I - beta K Lxx)(I - beta K Lyy), so one step is
 *     1. rho   = dt^2 (kappa * Lap_h u^n + f^n)            (5-point Laplacian)
 *     2. for every x-line j: (I - beta K Lxx) w = rho      (tridiagonal)
 *     3. for every y-line i: (I - beta K Lyy) d = w        (tridiagonal)
 *     4. u^{n+1} = 2 u^n - u^{n-1} + d
 *   Each tridiagonal system is solved by the textbook Thomas algorithm
 *   (Gaussian elimination without pivoting, stable here by strict diagonal
 *   dominance).  The paper solves the same systems by cyclic reduction; both
 *   give the same solution up to rounding.
 *
 *   Start-up, eq. (CN2): PAPER mode u^1 = u^0 + dt psi.  GHOST mode applies
 *   the step above at n = 0 with the ghost level u^{-1} = u^1 - 2 dt psi,
 *   which gives u^1 = u^0 + dt psi + e with
 *   (I - beta K Lxx)(I - beta K Lyy) e = (dt^2/2)(kappa Lap_h u^0 + f^0).
 *
 * Point sources add their value of f at one cell; receivers record u^{n+1}
 * at given cells after every step.  OpenMP only distributes independent
 * lines over threads; the arithmetic of every line is the sequential one.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)

/* Thomas algorithm for  a[k] x[k-1] + b[k] x[k] + c[k] x[k+1] = d[k],  k = 0..n-1
 * (a[0] and c[n-1] are ignored).  cp and dp are scratch arrays of n doubles.
 * Forward elimination computes the modified super-diagonal cp and right-hand
 * side dp; back substitution then gives x.  x may alias d. */
static void thomas(int n, const double *a, const double *b, const double *c,
                   const double *d, double *x, double *cp, double *dp)
{
    if (n <= 0) return;
    cp[0] = c[0] / b[0];
    dp[0] = d[0] / b[0];
    for (int k = 1; k < n; ++k) {
        double piv = b[k] - a[k] * cp[k - 1];
        cp[k] = c[k] / piv;
        dp[k] = (d[k] - a[k] * dp[k - 1]) / piv;
    }
    x[n - 1] = dp[n - 1];
    for (int k = n - 2; k >= 0; --k)
        x[k] = dp[k] - cp[k] * x[k + 1];
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* One tridiagonal solve, contiguous arrays. */
int oracle_thomas(int n, const double *a, const double *b, const double *c,
                  const double *d, double *x)
{
    if (n < 0) return ORACLE_EINVAL;
    if (n == 0) return ORACLE_OK;
    double *cp = malloc(sizeof(double) * (size_t)n);
    double *dp = malloc(sizeof(double) * (size_t)n);
    if (!cp || !dp) { free(cp); free(dp); return ORACLE_ENOMEM; }
    thomas(n, a, b, c, d, x, cp, dp);
    free(cp); free(dp);
    return ORACLE_OK;
}

/* Batch of independent systems.  Element k of system s sits at offset
 * s*sys_stride + k*elem_stride in every one of a, b, c, d; the solution
 * overwrites d. */
int oracle_tridiag_batched(int n, int batch, const double *a, const double *b,
                           const double *c, double *d, long long sys_stride,
                           long long elem_stride, int nthreads)
{
    if (n < 0 || batch < 0) return ORACLE_EINVAL;
    if (n == 0 || batch == 0) return ORACLE_OK;
    set_threads(nthreads);
    int err = 0;
#pragma omp parallel
    {
        double *buf = malloc(sizeof(double) * 6 * (size_t)n);
        if (!buf) {
#pragma omp atomic write
            err = 1;
        }
#pragma omp for schedule(static)
        for (int s = 0; s < batch; ++s) {
            if (!buf) continue;
            double *la = buf, *lb = buf + n, *lc = buf + 2 * n, *ld = buf + 3 * n;
            double *cp = buf + 4 * n, *dp = buf + 5 * n;
            for (int k = 0; k < n; ++k) {
                long long o = (long long)s * sys_stride + (long long)k * elem_stride;
                la[k] = a[o]; lb[k] = b[o]; lc[k] = c[o]; ld[k] = d[o];
            }
            thomas(n, la, lb, lc, ld, ld, cp, dp);
            for (int k = 0; k < n; ++k)
                d[(long long)s * sys_stride + (long long)k * elem_stride] = ld[k];
        }
        free(buf);
    }
    return err ? ORACLE_ENOMEM : ORACLE_OK;
}

/* rho = dt^2 (kappa * Lap_h u + f) on the interior, zero Dirichlet walls. */
static void assemble_rhs(int nx, int ny, double h, double dt, const double *kappa,
                         const double *u, const double *f, double *rho)
{
    const double inv_h2 = 1.0 / (h * h);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            size_t p = (size_t)j * nx + i;
            double uc = u[p];
            double uw = (i > 0) ? u[p - 1] : 0.0;
            double ue = (i < nx - 1) ? u[p + 1] : 0.0;
            double us = (j > 0) ? u[p - nx] : 0.0;
            double un = (j < ny - 1) ? u[p + nx] : 0.0;
            double lap = (uw - 2.0 * uc + ue) * inv_h2 + (us - 2.0 * uc + un) * inv_h2;
            rho[p] = dt * dt * (kappa[p] * lap + (f ? f[p] : 0.0));
        }
    }
}

/* Solve (I - beta K Lxx) w = rhs along every x-line (row j), then
 * (I - beta K Lyy) d = w along every y-line (column i).  On an x-line the
 * equation at node i reads
 *   -beta kappa_i / h^2 w_{i-1} + (1 + 2 beta kappa_i / h^2) w_i - beta kappa_i / h^2 w_{i+1} = rhs_i,
 * with w = 0 beyond the walls; y-lines likewise. */
static int adi_solves(int nx, int ny, double h, double dt, const double *kappa,
                      const double *rhs, double *w, double *d)
{
    const double beta = 0.5 * dt * dt;
    const double s = beta / (h * h);
    const int nmax = nx > ny ? nx : ny;
    int err = 0;
#pragma omp parallel
    {
        double *buf = malloc(sizeof(double) * 6 * (size_t)nmax);
        if (!buf) {
#pragma omp atomic write
            err = 1;
        }
        double *la = buf, *lb = buf + nmax, *lc = buf + 2 * nmax, *ld = buf + 3 * nmax;
        double *cp = buf + 4 * nmax, *dp = buf + 5 * nmax;
#pragma omp for schedule(static)
        for (int j = 0; j < ny; ++j) {
            if (!buf) continue;
            for (int i = 0; i < nx; ++i) {
                size_t p = (size_t)j * nx + i;
                double off = s * kappa[p];
                la[i] = -off; lb[i] = 1.0 + 2.0 * off; lc[i] = -off; ld[i] = rhs[p];
            }
            thomas(nx, la, lb, lc, ld, ld, cp, dp);
            memcpy(w + (size_t)j * nx, ld, sizeof(double) * (size_t)nx);
        }
#pragma omp for schedule(static)
        for (int i = 0; i < nx; ++i) {
            if (!buf) continue;
            for (int j = 0; j < ny; ++j) {
                size_t p = (size_t)j * nx + i;
                double off = s * kappa[p];
                la[j] = -off; lb[j] = 1.0 + 2.0 * off; lc[j] = -off; ld[j] = w[p];
            }
            thomas(ny, la, lb, lc, ld, ld, cp, dp);
            for (int j = 0; j < ny; ++j) d[(size_t)j * nx + i] = ld[j];
        }
        free(buf);
    }
    return err ? ORACLE_ENOMEM : ORACLE_OK;
}

/* f at level n from point sources: f[idx[s]] += amp[s]. */
static void scatter_sources(size_t npts, double *f, int nsrc, const int *idx,
                            const double *amp)
{
    memset(f, 0, sizeof(double) * npts);
    for (int s = 0; s < nsrc; ++s) f[idx[s]] += amp[s];
}

static int check_grid(int nx, int ny, double h, double dt)
{
    if (nx < 1 || ny < 1 || !(h > 0.0) || !(dt > 0.0)) return ORACLE_EINVAL;
    return ORACLE_OK;
}

/* One step from (u_prev, u_curr) with right-hand side source field f (may be
 * NULL), exposing the intermediates rho, w and d (each nx*ny, may be NULL),
 * writing u^{n+1} to u_next. */
int oracle_adi_step_parts(int nx, int ny, double h, double dt, const double *kappa,
                          const double *u_prev, const double *u_curr, const double *f,
                          double *rho_out, double *w_out, double *d_out,
                          double *u_next, int nthreads)
{
    if (check_grid(nx, ny, h, dt)) return ORACLE_EINVAL;
    set_threads(nthreads);
    size_t npts = (size_t)nx * ny;
    double *tmp = malloc(sizeof(double) * 3 * npts);
    if (!tmp) return ORACLE_ENOMEM;
    double *rho = tmp, *w = tmp + npts, *d = tmp + 2 * npts;
    assemble_rhs(nx, ny, h, dt, kappa, u_curr, f, rho);
    int rc = adi_solves(nx, ny, h, dt, kappa, rho, w, d);
    if (rc == ORACLE_OK) {
        for (size_t p = 0; p < npts; ++p)
            u_next[p] = 2.0 * u_curr[p] - u_prev[p] + d[p];
        if (rho_out) memcpy(rho_out, rho, sizeof(double) * npts);
        if (w_out) memcpy(w_out, w, sizeof(double) * npts);
        if (d_out) memcpy(d_out, d, sizeof(double) * npts);
    }
    free(tmp);
    return rc;
}

/* nsteps steps.  On entry u_prev, u_curr hold u^{n-1}, u^n; on return they
 * hold u^{n+nsteps-1}, u^{n+nsteps}.  Step k (0-based) uses the source values
 * src_amp[k*nsrc + s] at cells src_idx[s] and records u^{n+k+1} at cells
 * rec_idx[r] into traces[k*nrec + r].  nsrc / nrec may be 0 (arrays NULL). */
int oracle_adi_run(int nx, int ny, double h, double dt, const double *kappa,
                   double *u_prev, double *u_curr,
                   int nsrc, const int *src_idx, const double *src_amp,
                   int nrec, const int *rec_idx, double *traces,
                   int nsteps, int nthreads)
{
    if (check_grid(nx, ny, h, dt) || nsteps < 0 || nsrc < 0 || nrec < 0)
        return ORACLE_EINVAL;
    set_threads(nthreads);
    size_t npts = (size_t)nx * ny;
    for (int s = 0; s < nsrc; ++s)
        if (src_idx[s] < 0 || (size_t)src_idx[s] >= npts) return ORACLE_EINVAL;
    for (int r = 0; r < nrec; ++r)
        if (rec_idx[r] < 0 || (size_t)rec_idx[r] >= npts) return ORACLE_EINVAL;
    double *tmp = malloc(sizeof(double) * 4 * npts);
    if (!tmp) return ORACLE_ENOMEM;
    double *rho = tmp, *w = tmp + npts, *d = tmp + 2 * npts, *f = tmp + 3 * npts;
    int rc = ORACLE_OK;
    for (int k = 0; k < nsteps && rc == ORACLE_OK; ++k) {
        const double *fk = NULL;
        if (nsrc > 0) {
            scatter_sources(npts, f, nsrc, src_idx, src_amp + (size_t)k * nsrc);
            fk = f;
        }
        assemble_rhs(nx, ny, h, dt, kappa, u_curr, fk, rho);
        rc = adi_solves(nx, ny, h, dt, kappa, rho, w, d);
        if (rc != ORACLE_OK) break;
        /* u^{n+1} = 2u^n - u^{n-1} + d, then shift the two levels */
#pragma omp parallel for schedule(static)
        for (long long p = 0; p < (long long)npts; ++p) {
            double next = 2.0 * u_curr[p] - u_prev[p] + d[p];
            u_prev[p] = u_curr[p];
            u_curr[p] = next;
        }
        for (int r = 0; r < nrec; ++r)
            traces[(size_t)k * nrec + r] = u_curr[rec_idx[r]];
    }
    free(tmp);
    return rc;
}

/* Level u^1 from u^0, psi (NULL = 0) and the source values of level 0.
 * mode 0 = PAPER (u^1 = u^0 + dt psi, eq. (CN2)); mode 1 = GHOST (second order). */
int oracle_adi_start(int nx, int ny, double h, double dt, const double *kappa,
                     const double *u0, const double *psi, int nsrc,
                     const int *src_idx, const double *src_amp0, int mode,
                     double *u1, int nthreads)
{
    if (check_grid(nx, ny, h, dt) || nsrc < 0 || (mode != 0 && mode != 1))
        return ORACLE_EINVAL;
    set_threads(nthreads);
    size_t npts = (size_t)nx * ny;
    for (int s = 0; s < nsrc; ++s)
        if (src_idx[s] < 0 || (size_t)src_idx[s] >= npts) return ORACLE_EINVAL;
    if (mode == 0) {
        for (size_t p = 0; p < npts; ++p) u1[p] = u0[p] + dt * (psi ? psi[p] : 0.0);
        return ORACLE_OK;
    }
    double *tmp = malloc(sizeof(double) * 4 * npts);
    if (!tmp) return ORACLE_ENOMEM;
    double *rho = tmp, *w = tmp + npts, *e = tmp + 2 * npts, *f = tmp + 3 * npts;
    const double *fk = NULL;
    if (nsrc > 0) {
        scatter_sources(npts, f, nsrc, src_idx, src_amp0);
        fk = f;
    }
    assemble_rhs(nx, ny, h, dt, kappa, u0, fk, rho);
    for (size_t p = 0; p < npts; ++p) rho[p] *= 0.5;
    int rc = adi_solves(nx, ny, h, dt, kappa, rho, w, e);
    if (rc == ORACLE_OK)
        for (size_t p = 0; p < npts; ++p)
            u1[p] = u0[p] + dt * (psi ? psi[p] : 0.0) + e[p];
    free(tmp);
    return rc;
}

/* ------------------------------------------------------------------------
 * Discrete adjoint of oracle_adi_run (not in the paper; derived from the
 * scheme above).  With A_x = I - beta K Lxx, A_y = I - beta K Lyy, one step is
 *   u^{k+1} = 2u^k - u^{k-1} + A_y^{-1} A_x^{-1} dt^2 (K Lap u^k + f^k),
 * and the traces are tr_{k-1} = P u^{k+1} (P samples the receiver nodes).
 * For a scalar J of the traces with g^m = P^T dJ/dtr_{m-2}, the adjoint
 * levels lambda^m = dJ/du^m obey, backwards from lambda^{S+2} = 0:
 *   nu      = A_y^{-T} lambda^{k+1}       (transposed y-line solves)
 *   mu      = A_x^{-T} nu                 (transposed x-line solves)
 *   dJ/dkappa += dt^2 mu (Lap u^k) + beta mu (Lxx w^k) + beta nu (Lyy d^k)
 *   dJ/df^k    = dt^2 mu                  (at the source nodes)
 *   lambda^k = g^k + 2 lambda^{k+1} - lambda^{k+2} + dt^2 Lap(kappa mu)
 * where w^k, d^k are the forward intermediates of step k.  The initial levels
 * are taken as independent of kappa.  The transposed line systems are solved
 * by Thomas on the transposed coefficients (row i: -r_{i-1}, 1 + 2 r_i,
 * -r_{i+1}).  Everything is kept in memory: meant for small grids.
 * ------------------------------------------------------------------------ */
static void apply_lap(int nx, int ny, double h, const double *v, double *out)
{
    const double inv_h2 = 1.0 / (h * h);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t p = (size_t)j * nx + i;
            double c = v[p];
            double w_ = i > 0 ? v[p - 1] : 0.0, e_ = i < nx - 1 ? v[p + 1] : 0.0;
            double s_ = j > 0 ? v[p - nx] : 0.0, n_ = j < ny - 1 ? v[p + nx] : 0.0;
            out[p] = (w_ - 2.0 * c + e_) * inv_h2 + (s_ - 2.0 * c + n_) * inv_h2;
        }
}

static void apply_lxx(int nx, int ny, double h, const double *v, double *out)
{
    const double inv_h2 = 1.0 / (h * h);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t p = (size_t)j * nx + i;
            double w_ = i > 0 ? v[p - 1] : 0.0, e_ = i < nx - 1 ? v[p + 1] : 0.0;
            out[p] = (w_ - 2.0 * v[p] + e_) * inv_h2;
        }
}

static void apply_lyy(int nx, int ny, double h, const double *v, double *out)
{
    const double inv_h2 = 1.0 / (h * h);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t p = (size_t)j * nx + i;
            double s_ = j > 0 ? v[p - nx] : 0.0, n_ = j < ny - 1 ? v[p + nx] : 0.0;
            out[p] = (s_ - 2.0 * v[p] + n_) * inv_h2;
        }
}

/* ------------------------------------------------------------------------
 * Eq. (CN1) with a coefficient that changes in time (its c^{k+1} and c^{k-1}):
 * kappa_next multiplies the Laplacian of u^{k+1}, kappa_prev that of u^{k-1};
 * the coefficient at t_k does not enter.  With delta = u^{k+1} - 2u^k + u^{k-1}
 * and beta = dt^2 / 2, eq. (CN1) is
 *   (I - beta K+ Lap) delta = dt^2 f^k + beta (2 K+ Lap u^k + (K- - K+) Lap u^{k-1}),
 * and the ADI step replaces the operator on the left by
 * (I - beta K+ Lxx)(I - beta K+ Lyy), x-lines first.  With K- = K+ it is the
 * step of oracle_adi_step_parts.
 * ------------------------------------------------------------------------ */
int oracle_adi_step_tdc(int nx, int ny, double h, double dt, const double *kappa_prev,
                        const double *kappa_next, const double *u_prev, const double *u_curr,
                        const double *f, double *u_next, int nthreads)
{
    if (check_grid(nx, ny, h, dt)) return ORACLE_EINVAL;
    set_threads(nthreads);
    size_t npts = (size_t)nx * ny;
    double *tmp = malloc(sizeof(double) * 5 * npts);
    if (!tmp) return ORACLE_ENOMEM;
    double *lap_c = tmp, *lap_p = tmp + npts, *rho = tmp + 2 * npts;
    double *w = tmp + 3 * npts, *d = tmp + 4 * npts;
    const double beta = 0.5 * dt * dt;
    apply_lap(nx, ny, h, u_curr, lap_c);
    apply_lap(nx, ny, h, u_prev, lap_p);
    for (size_t p = 0; p < npts; ++p)
        rho[p] = dt * dt * (f ? f[p] : 0.0) +
                 beta * (2.0 * kappa_next[p] * lap_c[p] + (kappa_prev[p] - kappa_next[p]) * lap_p[p]);
    int rc = adi_solves(nx, ny, h, dt, kappa_next, rho, w, d);
    if (rc == ORACLE_OK)
        for (size_t p = 0; p < npts; ++p) u_next[p] = 2.0 * u_curr[p] - u_prev[p] + d[p];
    free(tmp);
    return rc;
}

/* ------------------------------------------------------------------------
 * The ADI split as printed, eqs. (fr1)-(fr2) (Sec. 2), and the line systems of
 * Listing 1 (Sec. 3.2).  Levels sit on half steps: the x-sub-step takes
 * (u^{k-1/2}, u^k) to u^{k+1/2}, the y-sub-step (u^k, u^{k+1/2}) to u^{k+1}.
 * Each sub-step is a three-level scheme with the tau^2 denominator and one
 * direction's second difference D (zero Dirichlet walls),
 *   (u_new - 2 u_mid + u_old) / tau^2 - th_new kappa D u_new - th_old kappa D u_old = f,
 * i.e. with g = th_new tau^2 kappa / h^2 the line system
 *   -g u_new[k-1] + (1 + 2 g) u_new[k] - g u_new[k+1]
 *      = 2 u_mid - u_old + th_old (tau^2 kappa / h^2) (u_old[k-1] - 2 u_old[k] + u_old[k+1]) + tau^2 f.
 * mode 1: eqs. (fr1)-(fr2): th_new = th_old = 1/2, f^k in the x-sub-step and
 *         f^{k+1/2} in the y-sub-step;
 * mode 2: Listing 1: a = c = tau^2, b = 2 tau^2 + h^2 and a right-hand side
 *         from the two older levels only, i.e. th_new = 1, th_old = 0 (the
 *         listing has kappa = 1 and f = 0; kappa and f enter as above).
 * ------------------------------------------------------------------------ */
static int split_substep(int nx, int ny, double h, double dt, const double *kappa, int along_y,
                         double th_new, double th_old, const double *u_old, const double *u_mid,
                         const double *f, double *u_new)
{
    const double s = dt * dt / (h * h);
    const int n = along_y ? ny : nx, lines = along_y ? nx : ny;
    const size_t step = along_y ? (size_t)nx : 1;
    int rc = ORACLE_OK;
#pragma omp parallel
    {
        double *buf = malloc(sizeof(double) * 6 * (size_t)n);
        if (!buf) {
#pragma omp atomic write
            rc = ORACLE_ENOMEM;
        } else {
            double *la = buf, *lb = buf + n, *lc = buf + 2 * n, *ld = buf + 3 * n;
            double *cp = buf + 4 * n, *dp = buf + 5 * n;
#pragma omp for schedule(static)
            for (int l = 0; l < lines; ++l) {
                for (int k = 0; k < n; ++k) {
                    size_t p = along_y ? (size_t)k * nx + l : (size_t)l * nx + k;
                    double lo = k > 0 ? u_old[p - step] : 0.0;
                    double hi = k < n - 1 ? u_old[p + step] : 0.0;
                    double g = th_new * s * kappa[p];
                    la[k] = k > 0 ? -g : 0.0;
                    lb[k] = 1.0 + 2.0 * g;
                    lc[k] = k < n - 1 ? -g : 0.0;
                    ld[k] = 2.0 * u_mid[p] - u_old[p] + th_old * s * kappa[p] * (lo - 2.0 * u_old[p] + hi) +
                            dt * dt * (f ? f[p] : 0.0);
                }
                thomas(n, la, lb, lc, ld, ld, cp, dp);
                for (int k = 0; k < n; ++k) {
                    size_t p = along_y ? (size_t)k * nx + l : (size_t)l * nx + k;
                    u_new[p] = ld[k];
                }
            }
            free(buf);
        }
    }
    return rc;
}

int oracle_adi_step_split(int nx, int ny, double h, double dt, const double *kappa, int mode,
                          const double *u_half, const double *u_curr, const double *f,
                          const double *f_half, double *u_half_next, double *u_next, int nthreads)
{
    if (check_grid(nx, ny, h, dt) || (mode != 1 && mode != 2)) return ORACLE_EINVAL;
    if (u_half_next == u_half || u_half_next == u_curr || u_next == u_half || u_next == u_curr ||
        u_next == u_half_next)
        return ORACLE_EINVAL;
    set_threads(nthreads);
    const double th_new = mode == 1 ? 0.5 : 1.0, th_old = mode == 1 ? 0.5 : 0.0;
    int rc = split_substep(nx, ny, h, dt, kappa, 0, th_new, th_old, u_half, u_curr, f, u_half_next);
    if (rc == ORACLE_OK)
        rc = split_substep(nx, ny, h, dt, kappa, 1, th_new, th_old, u_curr, u_half_next, f_half, u_next);
    return rc;
}

/* transposed line solves: along x (rows) or y (columns) */
static int transposed_solves(int nx, int ny, double h, double dt, const double *kappa,
                             int along_y, const double *rhs, double *out)
{
    const double s = 0.5 * dt * dt / (h * h);
    const int n = along_y ? ny : nx, lines = along_y ? nx : ny;
    double *buf = malloc(sizeof(double) * 6 * (size_t)n);
    if (!buf) return ORACLE_ENOMEM;
    double *la = buf, *lb = buf + n, *lc = buf + 2 * n, *ld = buf + 3 * n;
    double *cp = buf + 4 * n, *dp = buf + 5 * n;
    for (int l = 0; l < lines; ++l) {
        for (int k = 0; k < n; ++k) {
            size_t p = along_y ? (size_t)k * nx + l : (size_t)l * nx + k;
            size_t pm = along_y ? p - nx : p - 1, pp = along_y ? p + nx : p + 1;
            la[k] = k > 0 ? -s * kappa[pm] : 0.0;
            lb[k] = 1.0 + 2.0 * s * kappa[p];
            lc[k] = k < n - 1 ? -s * kappa[pp] : 0.0;
            ld[k] = rhs[p];
        }
        thomas(n, la, lb, lc, ld, ld, cp, dp);
        for (int k = 0; k < n; ++k) {
            size_t p = along_y ? (size_t)k * nx + l : (size_t)l * nx + k;
            out[p] = ld[k];
        }
    }
    free(buf);
    return ORACLE_OK;
}

int oracle_adjoint(int nx, int ny, double h, double dt, const double *kappa,
                   const double *u_prev0, const double *u_curr0,
                   int nsrc, const int *src_idx, const double *src_amp,
                   int nrec, const int *rec_idx, const double *grad_traces,
                   int nsteps, double *grad_kappa, double *grad_amp, int nthreads)
{
    if (check_grid(nx, ny, h, dt) || nsteps < 1 || nsrc < 0 || nrec < 0) return ORACLE_EINVAL;
    set_threads(nthreads);
    const size_t npts = (size_t)nx * ny;
    const double beta = 0.5 * dt * dt;
    const int S = nsteps;
    /* forward: levels U[0..S+1], x-sweep results W[1..S], increments D[1..S] */
    double *U = malloc(sizeof(double) * (size_t)(S + 2) * npts);
    double *W = malloc(sizeof(double) * (size_t)(S + 1) * npts);
    double *D = malloc(sizeof(double) * (size_t)(S + 1) * npts);
    double *tmp = malloc(sizeof(double) * 8 * npts);
    if (!U || !W || !D || !tmp) { free(U); free(W); free(D); free(tmp); return ORACLE_ENOMEM; }
    double *f = tmp, *rho = tmp + npts, *lam1 = tmp + 2 * npts, *lam2 = tmp + 3 * npts;
    double *nu = tmp + 4 * npts, *mu = tmp + 5 * npts, *a1 = tmp + 6 * npts, *a2 = tmp + 7 * npts;
    memcpy(U, u_prev0, sizeof(double) * npts);
    memcpy(U + npts, u_curr0, sizeof(double) * npts);
    int rc = ORACLE_OK;
    for (int k = 1; k <= S && rc == ORACLE_OK; ++k) {
        const double *fk = NULL;
        if (nsrc > 0) { scatter_sources(npts, f, nsrc, src_idx, src_amp + (size_t)(k - 1) * nsrc); fk = f; }
        assemble_rhs(nx, ny, h, dt, kappa, U + (size_t)k * npts, fk, rho);
        rc = adi_solves(nx, ny, h, dt, kappa, rho, W + (size_t)k * npts, D + (size_t)k * npts);
        for (size_t p = 0; p < npts; ++p)
            U[(size_t)(k + 1) * npts + p] = 2.0 * U[(size_t)k * npts + p] - U[(size_t)(k - 1) * npts + p] +
                                           D[(size_t)k * npts + p];
    }
    /* reverse */
    memset(grad_kappa, 0, sizeof(double) * npts);
    memset(lam2, 0, sizeof(double) * npts);             /* lambda^{k+2} */
    memset(lam1, 0, sizeof(double) * npts);             /* lambda^{k+1} */
    for (int r = 0; r < nrec; ++r) lam1[rec_idx[r]] += grad_traces[(size_t)(S - 1) * nrec + r];
    for (int k = S; k >= 1 && rc == ORACLE_OK; --k) {
        rc = transposed_solves(nx, ny, h, dt, kappa, 1, lam1, nu);
        if (rc == ORACLE_OK) rc = transposed_solves(nx, ny, h, dt, kappa, 0, nu, mu);
        if (rc != ORACLE_OK) break;
        apply_lap(nx, ny, h, U + (size_t)k * npts, a1);
        for (size_t p = 0; p < npts; ++p) grad_kappa[p] += dt * dt * mu[p] * a1[p];
        apply_lxx(nx, ny, h, W + (size_t)k * npts, a1);
        apply_lyy(nx, ny, h, D + (size_t)k * npts, a2);
        for (size_t p = 0; p < npts; ++p) grad_kappa[p] += beta * (mu[p] * a1[p] + nu[p] * a2[p]);
        if (grad_amp)
            for (int s = 0; s < nsrc; ++s) grad_amp[(size_t)(k - 1) * nsrc + s] = dt * dt * mu[src_idx[s]];
        /* lambda^k = g^k + 2 lambda^{k+1} - lambda^{k+2} + dt^2 Lap(kappa mu) */
        for (size_t p = 0; p < npts; ++p) a2[p] = kappa[p] * mu[p];
        apply_lap(nx, ny, h, a2, a1);
        for (size_t p = 0; p < npts; ++p) {
            double lk = 2.0 * lam1[p] - lam2[p] + dt * dt * a1[p];
            lam2[p] = lam1[p];
            lam1[p] = lk;
        }
        if (k >= 2)
            for (int r = 0; r < nrec; ++r) lam1[rec_idx[r]] += grad_traces[(size_t)(k - 2) * nrec + r];
    }
    free(U); free(W); free(D); free(tmp);
    return rc;
}
