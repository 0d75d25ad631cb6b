// cr.hpp -- the paper's line solver, cyclic reduction with one launch per level
// (Sec. 3.1: a forward-reduction kernel per level, one division for the last
// equation, a back-substitution kernel per level), rebuilt for all lines of a
// sweep at once: every launch covers every line of the grid, there are no
// per-line launches or host copies.  It is the same-GPU baseline for the
// partition solvers of the default step; included by adiwave.hip.
//
// A line of n unknowns (1-based i = 1..n) is treated as the first n of
// N = 2^m - 1 >= n equations, the rest being x_i = 0 (a = c = 0, b = 1, d = 0);
// they are never stored.  Forward level k (k = 1 .. m-1, h = 2^(k-1)) updates the
// equations at multiples of 2h from their neighbours i - h, i + h:
//     alpha = -a_i / b_{i-h},  gamma = -c_i / b_{i+h}
//     a_i <- alpha a_{i-h},  c_i <- gamma c_{i+h},
//     b_i <- b_i + alpha c_{i-h} + gamma a_{i+h},  d_i <- d_i + alpha d_{i-h} + gamma d_{i+h}.
// The equation left at 2^(m-1) gives x = d / b.  Back-substitution level k
// (k = m-1 .. 1) solves the odd multiples of h from the known x_{i-h}, x_{i+h}:
//     x_i = (d_i - a_i x_{i-h} - c_i x_{i+h}) / b_i,
// with the solution written over d.  Element (line l, index i) of every array is
// at l * ls + (i - 1) * es: x-lines ls = nx, es = 1; y-lines ls = 1, es = nx
// (consecutive lines of a y-sweep are adjacent columns, so its accesses coalesce).

namespace adw {

template <typename T>
struct CrArgs {
    T* a;
    T* b;
    T* c;
    T* d;
    int n, lines;
    long long ls, es;
    int h;            // half step of the level (2^(k-1))
};

// equation (line, i) with the virtual padding rows
template <typename T>
__device__ __forceinline__ void cr_load(const CrArgs<T>& A, int line, int i, T& a, T& b, T& c, T& d)
{
    if (i < 1 || i > A.n) { a = T(0); b = T(1); c = T(0); d = T(0); return; }
    const long long p = (long long)line * A.ls + (long long)(i - 1) * A.es;
    a = A.a[p]; b = A.b[p]; c = A.c[p]; d = A.d[p];
}

// forward level: equations at multiples of 2h (at most n / (2h) per line)
template <typename T>
__global__ void __launch_bounds__(256) k_cr_forward(CrArgs<T> A)
{
    const int per = A.n / (2 * A.h);
    const long long total = (long long)per * A.lines;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total; t += (long long)gridDim.x * 256) {
        // y-lines: neighbouring threads take neighbouring lines; x-lines: neighbouring equations
        const bool ymajor = A.ls == 1;
        const int line = ymajor ? (int)(t % A.lines) : (int)(t / per);
        const int q = ymajor ? (int)(t / A.lines) : (int)(t % per);
        const int i = (q + 1) * 2 * A.h;
        T a, b, c, d, a1, b1, c1, d1, a2, b2, c2, d2;
        cr_load(A, line, i, a, b, c, d);
        cr_load(A, line, i - A.h, a1, b1, c1, d1);
        cr_load(A, line, i + A.h, a2, b2, c2, d2);
        const T alpha = -a / b1;
        const T gamma = -c / b2;
        const long long p = (long long)line * A.ls + (long long)(i - 1) * A.es;
        A.a[p] = alpha * a1;
        A.c[p] = gamma * c2;
        A.b[p] = b + alpha * c1 + gamma * a2;
        A.d[p] = d + alpha * d1 + gamma * d2;
    }
}

// the single equation left at 2^(m-1) (h = 2^(m-1) here), solved in place
template <typename T>
__global__ void __launch_bounds__(256) k_cr_div(CrArgs<T> A)
{
    for (long long line = (long long)blockIdx.x * 256 + threadIdx.x; line < A.lines;
         line += (long long)gridDim.x * 256) {
        const int i = A.h;
        if (i > A.n) continue;
        const long long p = line * A.ls + (long long)(i - 1) * A.es;
        A.d[p] = A.d[p] / A.b[p];
    }
}

// back-substitution level: odd multiples of h
template <typename T>
__global__ void __launch_bounds__(256) k_cr_backward(CrArgs<T> A)
{
    const int per = (A.n / A.h + 1) / 2;
    const long long total = (long long)per * A.lines;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total; t += (long long)gridDim.x * 256) {
        const bool ymajor = A.ls == 1;
        const int line = ymajor ? (int)(t % A.lines) : (int)(t / per);
        const int q = ymajor ? (int)(t / A.lines) : (int)(t % per);
        const int i = (2 * q + 1) * A.h;
        const long long p = (long long)line * A.ls + (long long)(i - 1) * A.es;
        const T xl = (i - A.h >= 1) ? A.d[p - (long long)A.h * A.es] : T(0);
        const T xr = (i + A.h <= A.n) ? A.d[p + (long long)A.h * A.es] : T(0);
        A.d[p] = (A.d[p] - A.a[p] * xl - A.c[p] * xr) / A.b[p];
    }
}

// coefficients of the x- (dir 0) or y-lines (dir 1): -r, 1 + 2r, -r, without the
// couplings past the grid edge; for dir 0 also d = rho (5-point right-hand side,
// point sources of the step), for dir 1 d is left as it is (the x-sweep result)
template <typename T>
__global__ void __launch_bounds__(256) k_cr_setup(const T* __restrict__ u, const T* __restrict__ r, T* a, T* b,
                                                  T* c, T* d, int nx, int ny, int dir, T rho_scale)
{
    const long long n = (long long)nx * ny;
    for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < n; p += (long long)gridDim.x * 256) {
        const int j = (int)(p / nx), i = (int)(p - (long long)j * nx);
        const T rr = r[p];
        const bool first = dir == 0 ? i == 0 : j == 0;
        const bool last = dir == 0 ? i == nx - 1 : j == ny - 1;
        a[p] = first ? T(0) : -rr;
        c[p] = last ? T(0) : -rr;
        b[p] = T(1) + T(2) * rr;
        if (dir == 0) {
            const T uc = u[p];
            const T uw = i > 0 ? u[p - 1] : T(0), ue = i < nx - 1 ? u[p + 1] : T(0);
            const T us = j > 0 ? u[p - nx] : T(0), un = j < ny - 1 ? u[p + nx] : T(0);
            d[p] = rho_scale * (T(2) * rr * (((uw + ue) + (us + un)) - T(4) * uc));
        }
    }
}

// point sources of the step: d[idx] += rho_scale dt^2 amp (one thread, in order)
template <typename T>
__global__ void k_cr_sources(T* d, const int* __restrict__ idx, const T* __restrict__ amp, int count, T scale,
                             long long n)
{
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (int k = 0; k < count; ++k) {
            const int id = idx[k];
            if (id >= 0 && id < n) d[id] += scale * amp[k];
        }
}

// u_next = alpha u + beta v + d (v may be null when beta == 0)
template <typename T>
__global__ void __launch_bounds__(256) k_cr_update(const T* __restrict__ u, const T* v, const T* __restrict__ d,
                                                   T* out, T alpha, T beta, long long n)
{
    for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < n; p += (long long)gridDim.x * 256) {
        const T vv = v ? v[p] : T(0);
        out[p] = fma_rn(beta, vv, alpha * u[p]) + d[p];
    }
}

}  // namespace adw
