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
//   k_tri_part_iface2   the interface system, several threads per system (a
//                       second partition level in registers and LDS), writes X_p
//                       into d and into the workspace (k_tri_part_iface, one
//                       thread per system, for interface systems too long for it);
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

// The interface system in parallel: TPS threads per system (a power of two, 256 /
// TPS systems per workgroup), each owning a group of L <= kTpL consecutive interface
// rows.  The same partition once more, in registers and LDS: every group's last row
// carries a second-level unknown Z_i; the group's other rows are eliminated onto
// Z_{i-1} and Z_i, which leaves one equation per group (its Schur complement row),
// and these G <= TPS equations per system are solved by Thomas in LDS by one thread
// of the system.  Each thread then recovers its group's rows from Z_{i-1} and Z_i
// and writes them into slot 2 of the records and into d.  Lanes take neighbouring
// systems first, so the record rows load in runs of 256 / TPS values.
constexpr int kTpL = 16;            // interface rows per thread at most

template <typename T>
__global__ void __launch_bounds__(256) k_tri_part_iface2(TriArgs<T> A, int P, int M, int TPS, T* __restrict__ red)
{
    __shared__ T s_c[256];                         // C of each group's last row
    __shared__ T s_a[256], s_b[256], s_cc[256], s_d[256], s_z[256];   // second-level rows, Z
    const int spw = 256 / TPS;                     // systems per workgroup
    const int t = threadIdx.x;
    const int sl = t % spw, gi = t / spw;          // system in the workgroup, group
    const long long nb = A.batch;
    const long long s = (long long)blockIdx.x * spw + sl;
    const long long q = (long long)P * nb;
    const int L = (P + TPS - 1) / TPS;
    const int G = (P + L - 1) / L;                 // groups holding rows
    const int p0 = gi * L;
    const int np = (s < nb && gi < G) ? min(P, p0 + L) - p0 : 0;   // rows of the group
    const int li = np - 1;                         // interior rows (np - 1), -1 if none
    const int slot = sl * TPS + gi;                // this group's second-level row
    T ra[kTpL], rb[kTpL], rc[kTpL], rd[kTpL];
#pragma unroll
    for (int k = 0; k < kTpL; ++k) {
        if (k < np) {
            const T* g = red + (long long)(p0 + k) * nb + s;
            ra[k] = g[0];
            rb[k] = g[q] - g[3 * q];
            rc[k] = g[4 * q];
            rd[k] = g[2 * q] - g[5 * q];
        }
    }
    if (p0 == 0) ra[0] = T(0);
    // the group's last row (selected with static indices, so the arrays stay in registers)
    T ar = T(0), br = T(0), cr = T(0), dr = T(0);
#pragma unroll
    for (int k = 0; k < kTpL; ++k)
        if (k == li) { ar = ra[k]; br = rb[k]; cr = rc[k]; dr = rd[k]; }
    s_c[t] = cr;
    __syncthreads();
    const T cprv = (gi > 0 && np > 0) ? s_c[t - spw] : T(0);   // C of the previous group's last row
    // interior elimination: y, v, w (against D, A e_first, C e_last) at the first and
    // last interior rows; an empty interior gives the limit triples
    T yf = T(0), vf = T(0), wf = T(-1), yl = T(0), vl = T(-1), wl = T(0);
    if (li > 0) {
        T cprev = T(0), dprev = T(0), vprev = T(0);
        T ce[kTpL], de[kTpL], ve[kTpL];
#pragma unroll
        for (int k = 0; k < kTpL - 1; ++k) {
            if (k < li) {
                const T ak = ra[k];
                const T m = T(1) / (rb[k] - ak * cprev);
                const bool last = k == li - 1;
                if (last) wl = rc[k] * m;
                cprev = last ? T(0) : rc[k] * m;
                dprev = (rd[k] - ak * dprev) * m;
                vprev = (k == 0 ? ak : -ak * vprev) * m;
                ce[k] = cprev;
                de[k] = dprev;
                ve[k] = vprev;
            }
        }
        yl = dprev;
        vl = vprev;
        T y = yl, v = vl, w = wl;
#pragma unroll
        for (int k = kTpL - 3; k >= 0; --k) {
            if (k < li - 1) {
                y = de[k] - ce[k] * y;
                v = ve[k] - ce[k] * v;
                w = -ce[k] * w;
            }
        }
        yf = y;
        vf = v;
        wf = w;
    }
    // this group's Schur row, and the part of the previous group's row that comes
    // from this group's first interior row
    if (np > 0) {
        s_a[slot] = -ar * vl;
        s_b[slot] = br - ar * wl;
        s_d[slot] = dr - ar * yl;
        s_cc[slot] = T(0);
    }
    __syncthreads();
    if (np > 0 && gi > 0) {
        s_b[slot - 1] -= cprv * vf;
        s_cc[slot - 1] = -cprv * wf;
        s_d[slot - 1] -= cprv * yf;
    }
    __syncthreads();
    // second-level Thomas, one thread per system
    if (gi == 0 && s < nb) {
        const int base = sl * TPS;
        T cp = T(0), dp = T(0);
        for (int g = 0; g < G; ++g) {
            const T m = T(1) / (s_b[base + g] - s_a[base + g] * cp);
            cp = s_cc[base + g] * m;
            dp = (s_d[base + g] - s_a[base + g] * dp) * m;
            s_cc[base + g] = cp;
            s_z[base + g] = dp;
        }
        T z = dp;
        for (int g = G - 2; g >= 0; --g) {
            z = s_z[base + g] - s_cc[base + g] * z;
            s_z[base + g] = z;
        }
    }
    __syncthreads();
    if (np <= 0) return;
    const T zl = gi > 0 ? s_z[slot - 1] : T(0);
    const T zh = s_z[slot];
    // the group's rows: its last row is Z_i; the interior from Z_{i-1}, Z_i
    T x[kTpL];
    if (li > 0) {
        T cprev = T(0), dprev = zl;
        T ce[kTpL], de[kTpL];
#pragma unroll
        for (int k = 0; k < kTpL - 1; ++k) {
            if (k < li) {
                const T ak = ra[k];
                const T m = T(1) / (rb[k] - ak * cprev);
                const bool last = k == li - 1;
                const T dk = last ? rd[k] - rc[k] * zh : rd[k];
                cprev = last ? T(0) : rc[k] * m;
                dprev = (dk - ak * dprev) * m;
                ce[k] = cprev;
                de[k] = dprev;
            }
        }
        T xv = T(0);
#pragma unroll
        for (int k = kTpL - 2; k >= 0; --k) {
            if (k < li) {
                xv = de[k] - ce[k] * xv;
                x[k] = xv;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kTpL; ++k) {
        if (k < np) {
            const int p = p0 + k;
            const T xk = k == li ? zh : x[k];
            red[2 * q + (long long)p * nb + s] = xk;
            const int r = min(A.n, (p + 1) * M) - 1;
            A.d[s * A.sys_stride + (long long)r * A.elem_stride] = xk;
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
    hipLaunchKernelGGL((k_tri_part_reduce<T, M>), dim3(g1), dim3(256), 0, st, t, P, red);
    // threads per system for the parallel interface solve: the least power of two
    // whose groups of at most kTpL rows cover P (at most 64); longer interface
    // systems take the serial solve, one thread per system
    int tps = 1;
    while (tps < 64 && (long long)tps * kTpL < P) tps *= 2;
    if ((long long)tps * kTpL >= P) {
        const long long spw = 256 / tps;
        const unsigned g2 = (unsigned)((t.batch + spw - 1) / spw);
        hipLaunchKernelGGL((k_tri_part_iface2<T>), dim3(g2), dim3(256), 0, st, t, P, M, tps, red);
    } else {
        const unsigned g2 = (unsigned)((t.batch + kTpIfaceThreads - 1) / kTpIfaceThreads);
        hipLaunchKernelGGL((k_tri_part_iface<T>), dim3(g2), dim3(kTpIfaceThreads), 0, st, t, P, M, red);
    }
    hipLaunchKernelGGL((k_tri_part_expand<T, M>), dim3(g1), dim3(256), 0, st, t, P, (const T*)red);
}

}  // namespace adw
