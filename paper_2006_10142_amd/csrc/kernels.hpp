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
// interface unknown X_c is the last row; its interior the Lc - 1 rows above.
// Eliminating the interior with X_{c-1} and X_c left open gives
//   first interior value = Pf + Lf X_{c-1} + Rf X_c
//   last interior value  = Pl + Ll X_{c-1} + Rl X_c
// (P: data part; L, R: responses to the two interface values, r only).  The
// interface row (coefficients -rI, 1 + 2 rI, -rI, right-hand side wI) then reads
//   A_c X_{c-1} + B_c X_c + C_c X_{c+1} = D_c
//   A_c = -rI Ll_c,  B_c = 1 + 2 rI - rI Rl_c - rI Lf_{c+1},  C_c = -rI Rf_{c+1},
//   D_c = E_c + rI Pf_{c+1},  E_c = wI + rI Pl_c,
// the chunk c+1 terms being absent for the last chunk.  A, B, C and rI depend
// on r only and are built once; every step writes E and Pf.
//
// Summary planes are blocked by kPB columns so that one column block's whole
// interface system is contiguous: plane v, chunk c, column i at
//   v*K*nxp + ((i / kPB) * K + c) * kPB + i % kPB,   nxp = nx rounded up to kPB.
enum SumPlane { kPlaneA = 0, kPlaneB = 1, kPlaneC = 2, kPlaneRI = 3, kPlaneE = 4, kPlanePf = 5 };
constexpr int kSummaryPlanes = 6;

__host__ __device__ __forceinline__ size_t plane_at(int v, int c, int i, int K, int nxp)
{
    return (size_t)v * K * nxp + ((size_t)(i / kPB) * K + c) * kPB + (i % kPB);
}

template <typename T>
struct YArgs {
    const T* w;          // x-sweep result
    const T* r;
    int nx, ny, M, K, nxp;
    T* sum;              // summary planes (blocked, see above)
    T* X;                // K*nx interface values, index c*nx + i
    const T* u;          // update: out = alpha*u + beta*v + d
    const T* v;          // may be null when beta == 0
    T* out;
    T alpha, beta;
    T* tmp;              // create-time scratch for the static planes (5*K*nx)
    int rhs_times_r;     // right-hand side of the y-lines is r * w (adjoint solves)
};

// Data part of one chunk's interior elimination (top-down, pivots started
// afresh at the chunk): P forward value at the last interior row (Pl) and the
// first interior value of the P solution (Pf, as a running sum of
// prod_{i<k} q_i * forward_k).
template <typename T, bool FULL, int M>
__device__ __forceinline__ void ychunk_data(const T* __restrict__ wp, const T* __restrict__ rp,
                                            size_t nx, int L, T& Pf, T& Pl, bool scale)
{
    T q = T(0), dpv = T(0), pi = T(1), yP = T(0);
    for (int k = 0; k < (FULL ? M - 1 : L - 1); ++k) {
        const T rk = rp[(size_t)k * nx];
        const T wk = scale ? rk * wp[(size_t)k * nx] : wp[(size_t)k * nx];
        const T m = pivot_step<T>(rk, q);
        dpv = fma_rn(rk, dpv, wk) * m;
        yP = fma_rn(pi, dpv, yP);
        pi = pi * q;
    }
    Pf = yP;
    Pl = dpv;
}

// Unfused chunk reduction: one thread per (column, chunk) writes E and Pf.
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
    T Pf = T(0), Pl = T(0);
    const bool sc = A.rhs_times_r != 0;
    if (L == 16 && A.M == 16) ychunk_data<T, true, 16>(wp, rp, nx, L, Pf, Pl, sc);
    else if (L == 32 && A.M == 32) ychunk_data<T, true, 32>(wp, rp, nx, L, Pf, Pl, sc);
    else if (L >= 2) ychunk_data<T, false, 1>(wp, rp, nx, L, Pf, Pl, sc);
    const T rI = rp[(size_t)(L - 1) * nx];
    const T wI = sc ? rI * wp[(size_t)(L - 1) * nx] : wp[(size_t)(L - 1) * nx];
    A.sum[plane_at(kPlaneE, c, i, A.K, A.nxp)] = fma_rn(rI, Pl, wI);
    A.sum[plane_at(kPlanePf, c, i, A.K, A.nxp)] = Pf;
}

// Static planes, pass 1: the r-only responses of every chunk (Lf, Rf, Ll, Rl, rI)
// into A.tmp (5 planes of K*nx, index v*K*nx + c*nx + i).
template <typename T>
__global__ void __launch_bounds__(256) k_ystatic1(YArgs<T> A)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= A.nx) return;
    const size_t nx = (size_t)A.nx;
    const int lo = c * A.M;
    const int L = min(A.M, A.ny - lo);
    const T* __restrict__ rp = A.r + (size_t)lo * nx + i;
    T Lf = T(0), Rf = T(1), Ll = T(1), Rl = T(0);      // one-row chunk
    if (L >= 2) {
        T q = T(0), dlv = T(1), pi = T(1), yL = T(0);
        for (int k = 0; k < L - 1; ++k) {
            (void)pivot_step<T>(rp[(size_t)k * nx], q);
            dlv = q * dlv;                 // response to X_{c-1}: prod of q
            yL = fma_rn(pi, dlv, yL);
            pi = pi * q;
        }
        Lf = yL; Rf = pi; Ll = dlv; Rl = q;
    }
    const size_t plane = (size_t)A.K * nx;
    T* o = A.tmp + (size_t)c * nx + i;
    o[0 * plane] = Lf; o[1 * plane] = Rf; o[2 * plane] = Ll; o[3 * plane] = Rl;
    o[4 * plane] = rp[(size_t)(L - 1) * nx];
}

// Static planes, pass 2: interface-system coefficients A, B, C and rI.
template <typename T>
__global__ void __launch_bounds__(256) k_ystatic2(YArgs<T> A)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= A.nx) return;
    const size_t nx = (size_t)A.nx;
    const size_t plane = (size_t)A.K * nx;
    const T* t = A.tmp + (size_t)c * nx + i;
    const T Ll = t[2 * plane], Rl = t[3 * plane], rI = t[4 * plane];
    T nLf = T(0), nRf = T(0);
    if (c + 1 < A.K) { nLf = t[nx]; nRf = t[plane + nx]; }
    A.sum[plane_at(kPlaneA, c, i, A.K, A.nxp)] = (c == 0) ? T(0) : -rI * Ll;
    A.sum[plane_at(kPlaneB, c, i, A.K, A.nxp)] = T(1) + T(2) * rI - rI * Rl - rI * nLf;
    A.sum[plane_at(kPlaneC, c, i, A.K, A.nxp)] = -rI * nRf;
    A.sum[plane_at(kPlaneRI, c, i, A.K, A.nxp)] = rI;
}

// Interface system of every column, solved with the partition solver: a
// workgroup owns one block of kPB columns, P threads per column, SK consecutive
// chunks per thread.
template <typename T, int SK, int P>
__device__ __forceinline__ void yscan_block(const YArgs<T>& A, const int blk, T* lds)
{
    constexpr int CB = kPB;
    const int col = threadIdx.x % CB;
    const int t = threadIdx.x / CB;
    const int i = blk * CB + col;
    const bool live = i < A.nx;
    const int K = A.K;
    const int c0 = t * SK;
    const int L = live ? max(0, min(SK, K - c0)) : 0;
    const int nact = live ? (K + SK - 1) / SK : 0;
    const size_t pl = (size_t)K * A.nxp;
    const T* __restrict__ base = A.sum + ((size_t)blk * K) * kPB + col;

    T a[SK], b[SK], cc[SK], d[SK];
#pragma unroll
    for (int k = 0; k < SK; ++k) {
        a[k] = T(0); b[k] = T(1); cc[k] = T(0); d[k] = T(0);
        const int c = c0 + k;
        if (k < L) {
            const T* s = base + (size_t)c * kPB;
            a[k] = s[kPlaneA * pl];
            b[k] = s[kPlaneB * pl];
            cc[k] = s[kPlaneC * pl];
            const T nPf = (c + 1 < K) ? s[kPlanePf * pl + kPB] : T(0);
            d[k] = fma_rn(s[kPlaneRI * pl], nPf, s[kPlaneE * pl]);
        }
    }
    partition_solve<T, SK, P>(d, CoefABC<T, SK>{a, b, cc}, L, t, nact, lds + col, CB);
#pragma unroll
    for (int k = 0; k < SK; ++k)
        if (k < L) A.X[(size_t)(c0 + k) * A.nx + i] = d[k];
}

template <typename T, int SK, int P>
__global__ void __launch_bounds__(kPB * P) k_yscan(YArgs<T> A)
{
    __shared__ T lds[partition_lds_slots<P>() * kPB];
    yscan_block<T, SK, P>(A, blockIdx.x, lds);
}

// One thread per (column, chunk): the chunk's interior re-solved with X_{c-1}
// and X_c known, then the update out = alpha u + beta v + d of every row.
// Rows are loaded in groups of GR (a scheduling barrier between groups keeps
// the compiler from hoisting every load of the chunk, which would cost
// occupancy); FULL = the chunk has all M rows.
template <typename T, int M, int GR, bool FULL>
__device__ __forceinline__ void ysolve_chunk(const YArgs<T>& A, size_t base, size_t nx, int L, T Xp, T Xc)
{
    const T* __restrict__ w = A.w;
    const T* __restrict__ r = A.r;
    const T* __restrict__ u = A.u;
    const T* v = A.v;     // may be the same buffer as out (u^{n+1} written over u^{n-1})
    T* out = A.out;
    const bool scale = A.rhs_times_r != 0;
    T qa[M], da[M];
    T q = T(0), dpv = T(0);
#pragma unroll
    for (int g0 = 0; g0 < M - 1; g0 += GR) {
        T rr[GR], ww[GR];
#pragma unroll
        for (int k = g0; k < g0 + GR && k < M - 1; ++k) {
            rr[k - g0] = T(0); ww[k - g0] = T(0);
            if (FULL || k < L - 1) {
                rr[k - g0] = r[base + (size_t)k * nx];
                ww[k - g0] = __builtin_nontemporal_load(&w[base + (size_t)k * nx]);
                if (scale) ww[k - g0] *= rr[k - g0];
            }
        }
#pragma unroll
        for (int k = g0; k < g0 + GR && k < M - 1; ++k) {
            qa[k] = T(0); da[k] = T(0);
            if (FULL || k < L - 1) {
                const T rk = rr[k - g0];
                T rhs = ww[k - g0];
                if (k == 0) rhs = fma_rn(rk, Xp, rhs);
                const T m = pivot_step<T>(rk, q);
                dpv = fma_rn(rk, dpv, rhs) * m;
                qa[k] = q; da[k] = dpv;
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    const bool hasv = v != nullptr;
    const bool hasu = u != nullptr;
    T x = Xc;
#pragma unroll
    for (int g1 = M - 1; g1 >= 0; g1 -= GR) {
        T uu[GR], vv[GR];
#pragma unroll
        for (int k = g1; k > g1 - GR && k >= 0; --k) {
            uu[g1 - k] = T(0); vv[g1 - k] = T(0);
            if (FULL || k < L) {
                const size_t p = base + (size_t)k * nx;
                uu[g1 - k] = hasu ? u[p] : T(0);
                vv[g1 - k] = hasv ? __builtin_nontemporal_load(&v[p]) : T(0);
            }
        }
#pragma unroll
        for (int k = g1; k > g1 - GR && k >= 0; --k) {
            if (FULL || k < L) {
                if (k < L - 1) x = fma_rn(qa[k], x, da[k]);
                else x = Xc;
                __builtin_nontemporal_store(fma_rn(A.beta, vv[g1 - k], A.alpha * uu[g1 - k]) + x, &out[base + (size_t)k * nx]);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// column i, chunk c (i < nx)
template <typename T, int M, int GR>
__device__ __forceinline__ void ysolve_item(const YArgs<T>& A, const int i, const int c)
{
    const size_t nx = (size_t)A.nx;
    const int lo = c * M;
    const int L = min(M, A.ny - lo);
    const T Xp = (c > 0) ? A.X[(size_t)(c - 1) * nx + i] : T(0);
    const T Xc = A.X[(size_t)c * nx + i];
    const size_t base = (size_t)lo * nx + i;
    if (L == M) ysolve_chunk<T, M, GR, true>(A, base, nx, L, Xp, Xc);
    else ysolve_chunk<T, M, GR, false>(A, base, nx, L, Xp, Xc);
}

template <typename T, int M, int GR>
__global__ void __launch_bounds__(256) k_ysolve(YArgs<T> A)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < A.nx) ysolve_item<T, M, GR>(A, i, blockIdx.y);
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

// ------------------------------------------------------------------- copy ----
__global__ void __launch_bounds__(256) k_copy16(const float4* __restrict__ src, float4* __restrict__ dst,
                                                long long n)
{
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long step = (long long)gridDim.x * 256;
    for (; i < n; i += step) dst[i] = src[i];
}

}  // namespace adw
