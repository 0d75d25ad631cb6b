// tridiag_part.hpp -- the batched general line solve for layouts that the
// on-chip one-workgroup-per-system kernel does not take (strided elements,
// interleaved systems, very long lines).  It is a partition method in three
// launches, so that every unknown of every system keeps a thread busy instead
// of one thread walking a whole system; included by adiwave.hip.
//
// A system of n unknowns is cut into P = ceil(n/M) chunks of M rows.  The last
// row of chunk p holds its interface unknown X_p; the rows before it (the
// interior, at most M - 1) couple only to X_{p-1} (through a at the first
// interior row) and X_p (through c at the last one), so elimination expresses
// every interior unknown as
//     x_k = y_k - v_k X_{p-1} - w_k X_p,
// where y, v, w solve the interior matrix against d, a e_first and c e_last.
// Putting the interior rows next to each interface row into that row's equation
// leaves one tridiagonal equation per chunk in X_{p-1}, X_p, X_{p+1}: the Schur
// complement of the system onto the interface unknowns.  The Schur complement
// of a strictly diagonally dominant matrix is again strictly diagonally
// dominant, so plain elimination stays safe on it as on the full system.
//
//   k_tri_part_reduce   one thread per (system, chunk): interior elimination,
//                       then the interface equations' coefficients from the
//                       (y, v, w) at the first and last interior rows;
//   k_tri_part_iface    one thread per system: forms and solves the interface
//                       system, writes X_p into d and into the workspace;
//   k_tri_part_expand   one thread per (system, chunk): the interior again with
//                       X_{p-1}, X_p known, writes the interior of d.
// An empty interior (a chunk of one row) is the limit case: its first-row
// triple is (0, 0, -1) (that row is X_p itself) and its last-row triple
// (0, -1, 0) (the row before it is X_{p-1}).  Neighbouring threads take
// neighbouring systems, so interleaved systems (sys_stride 1) load whole lines.
// Workspace: 6 values per (chunk, system), slot q of record (p, s) at (q P + p) batch + s.

namespace adw {

constexpr int kTpM32 = 32;   // chunk rows, FP32 (4 (M-1) register values per thread)
constexpr int kTpM64 = 16;   // chunk rows, FP64

template <typename T, int M>
__device__ __forceinline__ int tp_load(const TriArgs<T>& A, long long s, int p, T (&ca)[M - 1], T (&cb)[M - 1],
                                       T (&cc)[M - 1], T (&cd)[M - 1], long long& base)
{
    const int k0 = p * M;
    const int li = min(A.n, k0 + M) - k0 - 1;
    const long long es = A.elem_stride;
    base = s * A.sys_stride + (long long)k0 * es;
#pragma unroll
    for (int i = 0; i < M - 1; ++i) {
        if (i < li) {
            const long long o = base + i * es;
            ca[i] = A.a[o];
            cb[i] = A.b[o];
            cc[i] = A.c[o];
            cd[i] = A.d[o];
        }
    }
    if (k0 == 0) ca[0] = T(0);          // a of the system's first row is not part of it
    return li;
}

// The interface row of chunk p is r = min(n, (p+1) M) - 1.  With primes for chunk
// p+1's first-row triple, its equation in X_{p-1}, X_p, X_{p+1} is
//   (-a_r v_l) X_{p-1} + (b_r - a_r w_l - c_r v'_f) X_p + (-c_r w'_f) X_{p+1}
//       = d_r - a_r y_l - c_r y'_f,
// with a_r = 0 for r = 0 and c_r = 0 on the last chunk.  The reduce launch writes
// it pre-combined, so that the serial solve reads six coalesced values a row:
// the thread of chunk p writes slots 0..2 of record p (-a_r v_l, b_r - a_r w_l,
// d_r - a_r y_l); the thread of chunk p+1 writes slots 3..5 of record p
// (c_r v'_f, -c_r w'_f, c_r y'_f), and the last chunk zeros its own.
template <typename T, int M>
__global__ void __launch_bounds__(256) k_tri_part_reduce(TriArgs<T> A, int P, T* __restrict__ red)
{
    const long long nb = A.batch;
    const long long gid = (long long)blockIdx.x * 256 + threadIdx.x;
    if (gid >= (long long)P * nb) return;
    const int p = (int)(gid / nb);
    const long long s = gid - (long long)p * nb;
    T ca[M - 1], cb[M - 1], cc[M - 1], cd[M - 1];
    long long base;
    const int li = tp_load<T, M>(A, s, p, ca, cb, cc, cd, base);
    // the chunk's interface row, and c of the row before the chunk
    const long long es = A.elem_stride;
    const int r = p * M + li;
    const long long orow = s * A.sys_stride + (long long)r * es;
    const T ar = r > 0 ? A.a[orow] : T(0);
    const T br = A.b[orow];
    const T dr = A.d[orow];
    const T cprv = p > 0 ? A.c[orow - (long long)(li + 1) * es] : T(0);
    T yf = T(0), vf = T(0), wf = T(-1), yl = T(0), vl = T(-1), wl = T(0);
    if (li > 0) {
        // forward elimination of the interior; c' over c, d' over d, v' over a
        T cprev = T(0), dprev = T(0), vprev = T(0);
#pragma unroll
        for (int i = 0; i < M - 1; ++i) {
            if (i < li) {
                const T ak = ca[i];
                const T m = T(1) / (cb[i] - ak * cprev);
                const bool last = i == li - 1;
                if (last) wl = cc[i] * m;
                cprev = last ? T(0) : cc[i] * m;
                dprev = (cd[i] - ak * dprev) * m;
                vprev = (i == 0 ? ak : -ak * vprev) * m;
                cc[i] = cprev;
                cd[i] = dprev;
                ca[i] = vprev;
            }
        }
        yl = dprev;
        vl = vprev;
        // back-substitution of the three columns up to the first interior row
        T y = yl, v = vl, w = wl;
#pragma unroll
        for (int i = M - 3; i >= 0; --i) {
            if (i < li - 1) {
                y = cd[i] - cc[i] * y;
                v = ca[i] - cc[i] * v;
                w = -cc[i] * w;
            }
        }
        yf = y;
        vf = v;
        wf = w;
    }
    const long long q = (long long)P * nb;
    T* o = red + (long long)p * nb + s;
    o[0] = -ar * vl;
    o[q] = br - ar * wl;
    o[2 * q] = dr - ar * yl;
    if (p > 0) {
        T* g = o - nb;                                       // record p - 1
        g[3 * q] = cprv * vf;
        g[4 * q] = -cprv * wf;
        g[5 * q] = cprv * yf;
    }
    if (p == P - 1) {
        o[3 * q] = T(0);
        o[4 * q] = T(0);
        o[5 * q] = T(0);
    }
}

// The recurrence is serial in p, but its loads are not: rows are fetched kTpAhead
// ahead into a register ring (static indices after unrolling), so that many
// loads of one thread are in flight at once.  Forward values go over slots 0 and 1
// of record p (read only at step p), the solution X_p into slot 2 and into d.
constexpr int kTpAhead = 4;         // 8 ahead, or 64-thread workgroups, measured slower
constexpr int kTpIfaceThreads = 256;

// the six raw values of a record; they are combined only where they are used, so
// that a prefetch does not wait for its own loads
template <typename T>
struct TpRow { T a, b, d, bc, c, dc; };

template <typename T>
__device__ __forceinline__ TpRow<T> tp_row(const T* red, long long s, int p, long long nb, long long q)
{
    const T* g = red + (long long)p * nb + s;
    return TpRow<T>{g[0], g[q], g[2 * q], g[3 * q], g[4 * q], g[5 * q]};
}

template <typename T>
__global__ void __launch_bounds__(kTpIfaceThreads) k_tri_part_iface(TriArgs<T> A, int P, int M, T* __restrict__ red)
{
    const long long s = (long long)blockIdx.x * kTpIfaceThreads + threadIdx.x;
    if (s >= A.batch) return;
    const long long nb = A.batch;
    const long long q = (long long)P * nb;
    T cprev = T(0), dprev = T(0);
    TpRow<T> ring[kTpAhead];
#pragma unroll
    for (int j = 0; j < kTpAhead; ++j)
        if (j < P) ring[j] = tp_row<T>(red, s, j, nb, q);
    for (int p0 = 0; p0 < P; p0 += kTpAhead) {
#pragma unroll
        for (int j = 0; j < kTpAhead; ++j) {
            const int p = p0 + j;
            if (p < P) {
                const TpRow<T> t = ring[j];
                if (p + kTpAhead < P) ring[j] = tp_row<T>(red, s, p + kTpAhead, nb, q);
                const T m = T(1) / ((t.b - t.bc) - t.a * cprev);
                cprev = t.c * m;
                dprev = ((t.d - t.dc) - t.a * dprev) * m;
                T* g = red + (long long)p * nb + s;
                g[0] = cprev;
                g[q] = dprev;
            }
        }
    }
    // back-substitution from the last chunk; (c', d') of chunk p fetched ahead too
    T x = dprev;
    T rc[kTpAhead], rd[kTpAhead];
#pragma unroll
    for (int j = 0; j < kTpAhead; ++j) {
        const int p = P - 2 - j;
        if (p >= 0) {
            const T* g = red + (long long)p * nb + s;
            rc[j] = g[0];
            rd[j] = g[q];
        }
    }
    {
        T* g = red + (long long)(P - 1) * nb + s;
        g[2 * q] = x;
        A.d[s * A.sys_stride + (long long)(A.n - 1) * A.elem_stride] = x;
    }
    for (int p0 = P - 2; p0 >= 0; p0 -= kTpAhead) {
#pragma unroll
        for (int j = 0; j < kTpAhead; ++j) {
            const int p = p0 - j;
            if (p >= 0) {
                x = rd[j] - rc[j] * x;
                const int pn = p - kTpAhead;
                if (pn >= 0) {
                    const T* gn = red + (long long)pn * nb + s;
                    rc[j] = gn[0];
                    rd[j] = gn[q];
                }
                T* g = red + (long long)p * nb + s;
                g[2 * q] = x;
                const int r = (p + 1) * M - 1;
                A.d[s * A.sys_stride + (long long)r * A.elem_stride] = x;
            }
        }
    }
}

template <typename T, int M>
__global__ void __launch_bounds__(256) k_tri_part_expand(TriArgs<T> A, int P, const T* __restrict__ red)
{
    const long long nb = A.batch;
    const long long gid = (long long)blockIdx.x * 256 + threadIdx.x;
    if (gid >= (long long)P * nb) return;
    const int p = (int)(gid / nb);
    const long long s = gid - (long long)p * nb;
    if (min(A.n, p * M + M) - p * M <= 1) return;          // no interior
    const long long q2 = 2 * (long long)P * nb;          // slot 2: X of each chunk
    const T xl = p > 0 ? red[q2 + (long long)(p - 1) * nb + s] : T(0);
    const T xh = red[q2 + (long long)p * nb + s];
    T ca[M - 1], cb[M - 1], cc[M - 1], cd[M - 1];
    long long base;
    const int li = tp_load<T, M>(A, s, p, ca, cb, cc, cd, base);
    // forward elimination with X_{p-1} folded into the first row, X_p into the last
    T cprev = T(0), dprev = xl;
#pragma unroll
    for (int i = 0; i < M - 1; ++i) {
        if (i < li) {
            const T ak = ca[i];
            const T m = T(1) / (cb[i] - ak * cprev);
            const bool last = i == li - 1;
            const T de = last ? cd[i] - cc[i] * xh : cd[i];
            cprev = last ? T(0) : cc[i] * m;
            dprev = (de - ak * dprev) * m;
            cc[i] = cprev;
            cd[i] = dprev;
        }
    }
    const long long es = A.elem_stride;
    T x = T(0);
#pragma unroll
    for (int i = M - 2; i >= 0; --i) {
        if (i < li) {
            x = cd[i] - cc[i] * x;
            A.d[base + i * es] = x;
        }
    }
}

// Workspace values the partition solve needs for (n, batch).
template <typename T>
size_t tri_part_workspace(int n, long long batch)
{
    const int M = sizeof(T) == 4 ? kTpM32 : kTpM64;
    return (size_t)6 * (size_t)((n + M - 1) / M) * (size_t)batch;
}

template <typename T>
void launch_tri_part(const TriArgs<T>& t, T* red, hipStream_t st)
{
    constexpr int M = sizeof(T) == 4 ? kTpM32 : kTpM64;
    const int P = (t.n + M - 1) / M;
    const long long work = (long long)P * t.batch;
    const unsigned g1 = (unsigned)((work + 255) / 256);
    const unsigned g2 = (unsigned)((t.batch + kTpIfaceThreads - 1) / kTpIfaceThreads);
    hipLaunchKernelGGL((k_tri_part_reduce<T, M>), dim3(g1), dim3(256), 0, st, t, P, red);
    hipLaunchKernelGGL((k_tri_part_iface<T>), dim3(g2), dim3(kTpIfaceThreads), 0, st, t, P, M, red);
    hipLaunchKernelGGL((k_tri_part_expand<T, M>), dim3(g1), dim3(256), 0, st, t, P, (const T*)red);
}

}  // namespace adw
