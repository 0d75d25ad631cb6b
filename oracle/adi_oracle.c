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
