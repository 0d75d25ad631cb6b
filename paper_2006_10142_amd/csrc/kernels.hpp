// kernels.hpp -- HIP kernels of one ADI step for gfx950 (wave64, 160 KiB LDS/CU).
//
// One step (the delta form of the Sec. 2 scheme, eq. (CN1) factored as in
// eqs. (fr1)-(fr2), x-lines first):
//   k_xsweep   rho = 2 r (5-point sum - 4 u) + dt^2 f, fused into the load of
//              u^n, then every x-line solved on chip -> w  (row strips; xsweep.hpp)
//   k_yreduce  every y-line cut into chunks of M rows; per chunk and column the
//              interior is eliminated top-down in one pass over w      (lane/column)
//   k_yscan    the chunk-interface system of every column (one unknown per
//              chunk), solved by the partition solver across threads
//   k_ysolve   every chunk re-solved with its two interface values known, fused
//              with u^{n+1} = 2u^n - u^{n-1} + d, written over u^{n-1}
// All lines are the tridiagonal systems  -r y_{k-1} + (1 + 2r) y_k - r y_{k+1}
// with r = dt^2 kappa / (2 h^2) of the node of row k.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "line_solver.hpp"
#include "xsweep.hpp"

namespace adw {

// ------------------------------------------------------------ vector access --
template <typename T> struct Vec16;
template <> struct Vec16<float> {
    using type = float4;
    static constexpr int N = 4;
    __device__ static void unpack(const float4& v, float* o) { o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w; }
    __device__ static float4 pack(const float* o) { return make_float4(o[0], o[1], o[2], o[3]); }
};
template <> struct Vec16<double> {
    using type = double2;
    static constexpr int N = 2;
    __device__ static void unpack(const double2& v, double* o) { o[0] = v.x; o[1] = v.y; }
    __device__ static double2 pack(const double* o) { return make_double2(o[0], o[1]); }
};

// Load the L <= S nodes of a segment starting at p (zeros beyond L).
// vec: p is 16-byte aligned for every segment with L == S.
template <typename T, int S>
__device__ __forceinline__ void load_seg(const T* __restrict__ p, int L, bool vec, T (&v)[S])
{
    using V = Vec16<T>;
    if constexpr (S % V::N == 0) {
        if (vec && L == S) {
            const typename V::type* q = reinterpret_cast<const typename V::type*>(p);
#pragma unroll
            for (int k = 0; k < S / V::N; ++k) V::unpack(q[k], &v[k * V::N]);
            return;
        }
    }
#pragma unroll
    for (int k = 0; k < S; ++k) v[k] = (k < L) ? p[k] : T(0);
}

template <typename T, int S>
__device__ __forceinline__ void store_seg(T* __restrict__ p, int L, bool vec, const T (&v)[S])
{
    using V = Vec16<T>;
    if constexpr (S % V::N == 0) {
        if (vec && L == S) {
            typename V::type* q = reinterpret_cast<typename V::type*>(p);
#pragma unroll
            for (int k = 0; k < S / V::N; ++k) q[k] = V::pack(&v[k * V::N]);
            return;
        }
    }
#pragma unroll
    for (int k = 0; k < S; ++k)
        if (k < L) p[k] = v[k];
}

// ------------------------------------------------------------- coefficient --
// r = s * speed^2 (speed field) or s * kappa (kappa field), s = dt^2 / (2 h^2).
template <typename T>
__global__ void __launch_bounds__(256) k_coef(const T* __restrict__ src, T scalar, int squared,
                                              T s, T* __restrict__ r, long long n)
{
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long step = (long long)gridDim.x * 256;
    for (; i < n; i += step) {
        T v = src ? src[i] : scalar;
        r[i] = squared ? s * (v * v) : s * v;
    }
}

// ---------------------------------------------------------------- y-lines ----
// Chunk c of a y-line covers rows [c*M, c*M + Lc), Lc = min(M, ny - c*M).  Its
// interface unknown is the last row; its interior the Lc - 1 rows above.
// Summary planes (each K*nx values, index c*nx + i):
//   0 Pf, 1 Lf, 2 Rf : first interior value = Pf + Lf X_{c-1} + Rf X_c
//   3 Pl, 4 Ll, 5 Rl : last interior value  = Pl + Ll X_{c-1} + Rl X_c
//   6 rI, 7 wI       : r and w of the interface row
constexpr int kSummaryPlanes = 8;

template <typename T>
struct YArgs {
    const T* w;          // x-sweep result
    const T* r;
    int nx, ny, M, K;
    T* sum;              // summary planes
    T* X;                // K*nx interface values
    const T* u;          // update: out = alpha*u + beta*v + d
    const T* v;          // may be null when beta == 0
    T* out;
    T alpha, beta;
    int nrec;            // receivers recorded from out after the update
    const int* rec_idx;
    T* traces;           // nrec values for this step
};

// One thread per (column, chunk): interior elimination streamed top-down.
// Interior rows k = 0..L-2 are eliminated with pivots started afresh at the
// chunk (q = 0); P = values with X_{c-1} = X_c = 0, L = response to X_{c-1},
// R = response to X_c.  First values come from the back-substitution written
// as a running sum (first = sum_k prod_{i<k} q_i * forward_k).
template <typename T, bool FULL>
__device__ __forceinline__ void yreduce_chunk(const T* __restrict__ wp, const T* __restrict__ rp,
                                              size_t nx, int L, T (&o)[8])
{
    T Pf = T(0), Lf = T(0), Rf = T(1), Pl = T(0), Ll = T(1), Rl = T(0);
    if (L >= 2) {
        T q = T(0), dpv = T(0), dlv = T(1), pi = T(1), yP = T(0), yL = T(0);
        for (int k = 0; k < (FULL ? 31 : L - 1); ++k) {
            const T rk = rp[(size_t)k * nx];
            const T wk = wp[(size_t)k * nx];
            const T m = pivot_step<T>(rk, q);
            dpv = fma_rn(rk, dpv, wk) * m;
            dlv = q * dlv;
            yP = fma_rn(pi, dpv, yP);
            yL = fma_rn(pi, dlv, yL);
            pi = pi * q;
        }
        Pf = yP; Lf = yL; Rf = pi;
        Pl = dpv; Ll = dlv; Rl = q;
    }
    o[0] = Pf; o[1] = Lf; o[2] = Rf; o[3] = Pl; o[4] = Ll; o[5] = Rl;
    o[6] = rp[(size_t)(L - 1) * nx];
    o[7] = wp[(size_t)(L - 1) * nx];
}

template <typename T>
__global__ void __launch_bounds__(256) k_yreduce(YArgs<T> A)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= A.nx) return;
    const size_t nx = (size_t)A.nx;
    const int lo = c * A.M;
    const int L = min(A.M, A.ny - lo);
    const T* __restrict__ wp = A.w + (size_t)lo * nx + i;
    const T* __restrict__ rp = A.r + (size_t)lo * nx + i;
    T o[8];
    if (L == 32 && A.M == 32) yreduce_chunk<T, true>(wp, rp, nx, L, o);
    else yreduce_chunk<T, false>(wp, rp, nx, L, o);
    const size_t plane = (size_t)A.K * nx;
    T* __restrict__ out = A.sum + (size_t)c * nx + i;
#pragma unroll
    for (int v = 0; v < kSummaryPlanes; ++v) out[v * plane] = o[v];
}

// Chunk-interface system of every column, solved with the partition solver:
// CB columns per workgroup, P threads per column, SK consecutive chunks per
// thread.  The equation of chunk c (interface row coefficients -rI, 1+2rI, -rI):
//   A_c = -rI Ll_c, B_c = 1 + 2rI - rI Rl_c - rI Lf_{c+1}, C_c = -rI Rf_{c+1},
//   D_c = wI + rI Pl_c + rI Pf_{c+1}      (terms of chunk c+1 absent for the last)
template <typename T, int SK, int P>
__global__ void __launch_bounds__(256) k_yscan(YArgs<T> A)
{
    constexpr int CB = 256 / P;
    __shared__ T lds[partition_lds_slots<P>() * CB];
    const int col = threadIdx.x % CB;
    const int t = threadIdx.x / CB;
    const int i = blockIdx.x * CB + col;
    const bool live = i < A.nx;
    const int K = A.K;
    const size_t nx = (size_t)A.nx;
    const size_t plane = (size_t)K * nx;
    const int c0 = t * SK;
    const int L = live ? max(0, min(SK, K - c0)) : 0;
    const int nact = live ? (K + SK - 1) / SK : 0;

    T a[SK], b[SK], cc[SK], d[SK];
#pragma unroll
    for (int k = 0; k < SK; ++k) {
        a[k] = T(0); b[k] = T(1); cc[k] = T(0); d[k] = T(0);
        const int c = c0 + k;
        if (k < L) {
            const T* s = A.sum + (size_t)c * nx + i;
            const T Pl = s[3 * plane], Ll = s[4 * plane], Rl = s[5 * plane];
            const T rI = s[6 * plane], wI = s[7 * plane];
            T nPf = T(0), nLf = T(0), nRf = T(0);
            if (c + 1 < K) {
                const T* sn = s + nx;
                nPf = sn[0]; nLf = sn[plane]; nRf = sn[2 * plane];
            }
            a[k] = -rI * Ll;
            b[k] = T(1) + T(2) * rI - rI * Rl - rI * nLf;
            cc[k] = -rI * nRf;
            d[k] = wI + rI * Pl + rI * nPf;
        }
    }
    partition_solve<T, SK, P>(d, CoefABC<T, SK>{a, b, cc}, L, t, nact, lds + col, CB);
#pragma unroll
    for (int k = 0; k < SK; ++k)
        if (k < L) A.X[(size_t)(c0 + k) * nx + i] = d[k];
}

// One thread per (column, chunk): the chunk's interior re-solved with X_{c-1}
// and X_c known, then the update out = alpha u + beta v + d of every row.
template <typename T, int M, bool FULL>
__device__ __forceinline__ void ysolve_chunk(const YArgs<T>& A, size_t base, size_t nx, int L, T Xp, T Xc)
{
    const T* __restrict__ w = A.w;
    const T* __restrict__ r = A.r;
    const T* __restrict__ u = A.u;
    const T* __restrict__ v = A.v;
    T* __restrict__ out = A.out;
    T qa[M], da[M];
    T q = T(0), dpv = T(0);
#pragma unroll
    for (int k = 0; k < M - 1; ++k) {
        qa[k] = T(0); da[k] = T(0);
        if (FULL || k < L - 1) {
            const T rk = r[base + (size_t)k * nx];
            T rhs = w[base + (size_t)k * nx];
            if (k == 0) rhs = fma_rn(rk, Xp, rhs);
            const T m = pivot_step<T>(rk, q);
            dpv = fma_rn(rk, dpv, rhs) * m;
            qa[k] = q; da[k] = dpv;
        }
    }
    const bool hasv = v != nullptr;
    {
        const size_t p = base + (size_t)(L - 1) * nx;
        const T vv = hasv ? v[p] : T(0);
        out[p] = fma_rn(A.beta, vv, A.alpha * u[p]) + Xc;
    }
    T x = Xc;
#pragma unroll
    for (int k = M - 2; k >= 0; --k) {
        if (FULL || k < L - 1) {
            x = fma_rn(qa[k], x, da[k]);
            const size_t p = base + (size_t)k * nx;
            const T vv = hasv ? v[p] : T(0);
            out[p] = fma_rn(A.beta, vv, A.alpha * u[p]) + x;
        }
    }
}

template <typename T, int M>
__global__ void __launch_bounds__(256) k_ysolve(YArgs<T> A)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= A.nx) return;
    const size_t nx = (size_t)A.nx;
    const int lo = c * M;
    const int L = min(M, A.ny - lo);
    const T Xp = (c > 0) ? A.X[(size_t)(c - 1) * nx + i] : T(0);
    const T Xc = A.X[(size_t)c * nx + i];
    const size_t base = (size_t)lo * nx + i;
    if (L == M) ysolve_chunk<T, M, true>(A, base, nx, L, Xp, Xc);
    else ysolve_chunk<T, M, false>(A, base, nx, L, Xp, Xc);
}

// traces[r] = out[idx[r]]; an offset outside [0, npts) records NaN
template <typename T>
__global__ void __launch_bounds__(256) k_record(const T* __restrict__ u, const int* __restrict__ idx,
                                                T* __restrict__ traces, int n, long long npts)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k < n) {
        const int id = idx[k];
        traces[k] = (id >= 0 && id < npts) ? u[id] : T(NAN);
    }
}

// u1 = u0 + dt psi (eq. (CN2))
template <typename T>
__global__ void __launch_bounds__(256) k_start_paper(const T* __restrict__ u0, const T* __restrict__ psi,
                                                     T dt, T* __restrict__ u1, long long n)
{
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long step = (long long)gridDim.x * 256;
    for (; i < n; i += step) u1[i] = u0[i] + (psi ? dt * psi[i] : T(0));
}

// ------------------------------------------------------ batched line solve ---
template <typename T>
struct TriArgs {
    const T* a; const T* b; const T* c; T* d;
    int n, batch;
    long long sys_stride, elem_stride;
    int vec;
    T* scratch;          // per-thread path: batch * n values
};

// One workgroup (TR threads) per contiguous system, nodes in registers.
template <typename T, int S, int TR>
__global__ void __launch_bounds__(TR >= 256 ? TR : 256) k_tridiag_wg(TriArgs<T> A)
{
    constexpr int NT = TR >= 256 ? TR : 256;
    constexpr int G = NT / TR;
    __shared__ T lds_all[G * partition_lds_slots<TR>()];
    const int g = threadIdx.x / TR;
    const int t = threadIdx.x - g * TR;
    const long long sys = (long long)blockIdx.x * G + g;
    const bool live = sys < A.batch;
    const int lo = t * S;
    const int L = live ? max(0, min(S, A.n - lo)) : 0;
    const int nact = live ? (A.n + S - 1) / S : 0;
    const long long off = (live ? sys : 0) * A.sys_stride + lo;
    const bool vec = A.vec != 0;
    T a[S], b[S], c[S], d[S];
    load_seg<T, S>(A.a + off, L, vec, a);
    load_seg<T, S>(A.b + off, L, vec, b);
    load_seg<T, S>(A.c + off, L, vec, c);
    load_seg<T, S>(A.d + off, L, vec, d);
#pragma unroll
    for (int k = 0; k < S; ++k) if (k >= L) b[k] = T(1);
    partition_solve<T, S, TR>(d, CoefABC<T, S>{a, b, c}, L, t, nact, lds_all + g * partition_lds_slots<TR>(), 1);
    if (L > 0) store_seg<T, S>(A.d + off, L, vec, d);
}

// One thread per system, any strides (Thomas with a global scratch row).
template <typename T>
__global__ void __launch_bounds__(256) k_tridiag_thread(TriArgs<T> A)
{
    const long long s = (long long)blockIdx.x * 256 + threadIdx.x;
    if (s >= A.batch) return;
    const long long es = A.elem_stride;
    const T* a = A.a + s * A.sys_stride;
    const T* b = A.b + s * A.sys_stride;
    const T* c = A.c + s * A.sys_stride;
    T* d = A.d + s * A.sys_stride;
    // scratch laid out [k][s] so that neighbouring threads touch neighbouring words
    T* cp = A.scratch + s;
    const long long cs = A.batch;
    T m = T(1) / b[0];
    T cpv = c[0] * m;
    T dpv = d[0] * m;
    cp[0] = cpv;
    d[0] = dpv;
    for (int k = 1; k < A.n; ++k) {
        const T ak = a[k * es];
        m = T(1) / (b[k * es] - ak * cpv);
        cpv = c[k * es] * m;
        dpv = (d[k * es] - ak * dpv) * m;
        cp[k * cs] = cpv;
        d[k * es] = dpv;
    }
    T x = dpv;
    for (int k = A.n - 2; k >= 0; --k) {
        x = d[k * es] - cp[k * cs] * x;
        d[k * es] = x;
    }
}

// ------------------------------------------------------------------- copy ----
__global__ void __launch_bounds__(256) k_copy16(const float4* __restrict__ src, float4* __restrict__ dst,
                                                long long n)
{
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long step = (long long)gridDim.x * 256;
    for (; i < n; i += step) dst[i] = src[i];
}

}  // namespace adw
