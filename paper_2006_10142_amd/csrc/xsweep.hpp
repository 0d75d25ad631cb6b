// xsweep.hpp -- x-lines of the ADI step on gfx950: right-hand side assembly
// fused into the load of u^n, an exact on-chip solve of every x-line, and
// (optionally) the first half of the y-line chunk elimination on the result.
//
// Line system of row j (Sec. 2, the x-implicit sub-step of eqs. (fr1)-(fr2)):
//     -r_i w_{i-1} + (1 + 2 r_i) w_i - r_i w_{i+1} = rho_i,   i = 0..nx-1,
// with rho = 2 r (u_W + u_E + u_S + u_N - 4 u_C) + dt^2 f  (eq. (CN1) in delta form).
//
// Elimination without pivoting (Thomas) in "q" form, q_i = -(modified super-diagonal):
//     m_i = 1 / (1 + r_i (2 - q_{i-1})),   q_i = r_i m_i,          q_{-1} = 0
//     g_i = m_i rho_i + q_i g_{i-1}                                 (forward)
//     w_i = g_i + q_i w_{i+1}                                       (backward)
// The pivots q depend on r only, which is fixed for the handle, so the pivot
// entering each 8-node segment is computed once (k_xpivots) and kept.  With it,
// a segment rebuilds its exact pivots locally and both recurrences become affine
// maps of the value carried in from the neighbouring segment:
//     g_out   = Gl + Ql g_in               (Gl: g with g_in = 0, Ql = prod q)
//     w_first = H + E g_in + Ql w_below    (H = sum P_e G_e, E = sum P_e Q_e,
//                                           P_e = prod_{i<e} q_i)
// A line is therefore solved by one forward and one backward scan of affine
// maps across its segments: DPP row shifts / broadcasts inside a wavefront, one
// LDS exchange across wavefronts -- the Thomas solution up to rounding.
//
// Layout: thread t of a line group owns nodes [8t, 8t+8) of the row (two
// 16-byte vectors); consecutive lanes read consecutive 32-byte blocks.
#pragma once
#include <hip/hip_runtime.h>

namespace adw {

// Reciprocal refined by Newton-Raphson steps y <- y + y (1 - x y) from the
// hardware estimate (one step for FP32, two for FP64).
__device__ __forceinline__ float nr_rcp(float x)
{
    float y = __builtin_amdgcn_rcpf(x);
    float e = __builtin_fmaf(-x, y, 1.0f);
    return __builtin_fmaf(e, y, y);
}
__device__ __forceinline__ double nr_rcp(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, y, 1.0);
    y = __builtin_fma(e, y, y);
    e = __builtin_fma(-x, y, 1.0);
    return __builtin_fma(e, y, y);
}
__device__ __forceinline__ float mul_rn(float a, float b) { return __fmul_rn(a, b); }
__device__ __forceinline__ double mul_rn(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ float fma_rn(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_rn(double a, double b, double c) { return __builtin_fma(a, b, c); }

// One elimination step of -r, 1+2r, -r rows: returns m, updates q in place.
// The same expression is used wherever a pivot sequence is built, so the
// pivots of a segment rebuilt from its stored entry value match a sweep over
// the whole line bit for bit.
template <typename T>
__device__ __forceinline__ T pivot_step(T r, T& q)
{
    const T m = nr_rcp(fma_rn(r, T(2) - q, T(1)));
    q = mul_rn(r, m);
    return m;
}

// ------------------------------------------------------------------ DPP ----
// GFX9 data-parallel-primitive controls used below
constexpr int kRowShr = 0x110;     // + n: shift right by n within a row of 16 lanes
constexpr int kRowShl = 0x100;     // + n: shift left by n within a row
constexpr int kWaveShr1 = 0x138;   // whole wavefront right by one lane
constexpr int kWaveShl1 = 0x130;   // whole wavefront left by one lane
constexpr int kRowBcast15 = 0x142; // lane 15 of each row to the next row
constexpr int kRowBcast31 = 0x143; // lane 31 to rows 2 and 3

// dpp<CTRL, ROWMASK>(old, src): src moved by the DPP pattern; lanes without a
// source (or in rows outside ROWMASK) receive `old`.
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ float dpp(float old, float src)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                                __builtin_bit_cast(int, src),
                                                                CTRL, ROWMASK, 0xf, false));
}
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ double dpp(double old, double src)
{
    const long long o = __builtin_bit_cast(long long, old), s = __builtin_bit_cast(long long, src);
    const int lo = __builtin_amdgcn_update_dpp((int)o, (int)s, CTRL, ROWMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(s >> 32), CTRL, ROWMASK, 0xf, false);
    return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ float readlane(float v, int l)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double readlane(double v, int l)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Affine maps x -> a + b x.  Forward scans compose a lane with earlier lanes,
// backward scans with later lanes; in both cases the lane's own map is applied
// last: (a, b) o (a2, b2) = (a + b a2, b b2).  Identity: (0, 1).
template <int CTRL, int ROWMASK, typename T>
__device__ __forceinline__ void compose_dpp(T& a, T& b)
{
    const T a2 = dpp<CTRL, ROWMASK>(T(0), a);
    const T b2 = dpp<CTRL, ROWMASK>(T(1), b);
    a = fma_rn(b, a2, a);
    b = b * b2;
}

// inclusive prefix (lanes 0..l) over the wavefront
template <typename T>
__device__ __forceinline__ void wave_scan_fwd(T& a, T& b)
{
    compose_dpp<kRowShr + 1, 0xf>(a, b);
    compose_dpp<kRowShr + 2, 0xf>(a, b);
    compose_dpp<kRowShr + 4, 0xf>(a, b);
    compose_dpp<kRowShr + 8, 0xf>(a, b);
    compose_dpp<kRowBcast15, 0xa>(a, b);
    compose_dpp<kRowBcast31, 0xc>(a, b);
}

// inclusive suffix (lanes l..63) over the wavefront
template <typename T>
__device__ __forceinline__ void wave_scan_bwd(T& a, T& b, int lane)
{
    compose_dpp<kRowShl + 1, 0xf>(a, b);
    compose_dpp<kRowShl + 2, 0xf>(a, b);
    compose_dpp<kRowShl + 4, 0xf>(a, b);
    compose_dpp<kRowShl + 8, 0xf>(a, b);
    // rows of 16 now hold row-local suffixes; fold in the rows above
    const T a16 = readlane(a, 16), b16 = readlane(b, 16);
    const T a32 = readlane(a, 32), b32 = readlane(b, 32);
    const T a48 = readlane(a, 48), b48 = readlane(b, 48);
    const T a23 = fma_rn(b32, a48, a32), b23 = b32 * b48;        // rows 2,3
    const T a13 = fma_rn(b16, a23, a16), b13 = b16 * b23;        // rows 1..3
    T ca = T(0), cb = T(1);
    if (lane < 16) { ca = a13; cb = b13; }
    else if (lane < 32) { ca = a23; cb = b23; }
    else if (lane < 48) { ca = a48; cb = b48; }
    a = fma_rn(b, ca, a);
    b = b * cb;
}

template <typename T>
struct XArgs {
    const T* u;          // u^n, (ny, nx)
    const T* r;          // r, (ny, nx)
    const T* qin;        // pivot entering each 8-node segment, (ny, nseg)
    T* w;                // out, (ny, nx)
    int nx, ny, nseg;    // nseg = ceil(nx / 8)
    int rows_per_strip;  // consecutive rows handled by one line group
    int vec;             // rows are 16-byte aligned and nx % 8 == 0
    T rho_scale;         // 1 for a step, 1/2 for the ghost start
    T tau2;              // dt^2
    int nsrc;            // point sources of this step
    const int* src_idx;
    const T* src_amp;    // nsrc values of f
    // fused y-chunk elimination: a strip is a whole number of y-chunks of M rows
    T* sum;              // summary planes (blocked by 16 columns, see kernels.hpp)
    int K, M, nxp;
};

constexpr int kSeg = 8;   // nodes per x-line segment (one segment per thread)
constexpr int kPB = 16;   // column block width of the y-chunk summary planes

// pivot entering every segment of every row: one thread per row, sequential
template <typename T>
__global__ void __launch_bounds__(256) k_xpivots(const T* __restrict__ r, T* __restrict__ qin,
                                                 int nx, int ny, int nseg)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= ny) return;
    const T* rr = r + (size_t)j * nx;
    T* qo = qin + (size_t)j * nseg;
    T q = T(0);
    for (int s = 0; s < nseg; ++s) {
        qo[s] = q;
        for (int e = 0; e < kSeg; ++e) {
            const int i = kSeg * s + e;
            if (i < nx) (void)pivot_step<T>(rr[i], q);
        }
    }
}

template <typename T>
__device__ __forceinline__ void load8(const T* __restrict__ row, int i0, int nx, bool vec, T (&v)[kSeg])
{
    if (vec && i0 + kSeg <= nx) {
        if constexpr (sizeof(T) == 4) {
            const float4 x = *reinterpret_cast<const float4*>(row + i0);
            const float4 y = *reinterpret_cast<const float4*>(row + i0 + 4);
            v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
            v[4] = y.x; v[5] = y.y; v[6] = y.z; v[7] = y.w;
        } else {
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const double2 x = *reinterpret_cast<const double2*>(row + i0 + 2 * h);
                v[2 * h] = x.x; v[2 * h + 1] = x.y;
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < kSeg; ++e) v[e] = (i0 + e < nx) ? row[i0 + e] : T(0);
    }
}

template <typename T>
__device__ __forceinline__ void store8(T* __restrict__ row, int i0, int nx, bool vec, const T (&v)[kSeg])
{
    if (vec && i0 + kSeg <= nx) {
        if constexpr (sizeof(T) == 4) {
            *reinterpret_cast<float4*>(row + i0) = make_float4(v[0], v[1], v[2], v[3]);
            *reinterpret_cast<float4*>(row + i0 + 4) = make_float4(v[4], v[5], v[6], v[7]);
        } else {
#pragma unroll
            for (int h = 0; h < 4; ++h)
                *reinterpret_cast<double2*>(row + i0 + 2 * h) = make_double2(v[2 * h], v[2 * h + 1]);
        }
    } else {
#pragma unroll
        for (int e = 0; e < kSeg; ++e)
            if (i0 + e < nx) row[i0 + e] = v[e];
    }
}

// Workgroup: max(TR, 256) threads = G line groups of TR threads.  A group owns
// rows_per_strip consecutive rows and solves them in turn; rows j+2 (u) and
// j+1 (r, entry pivots) are loaded while row j is being solved.
//
// FUSE: a strip is a whole number of y-chunks (rows_per_strip a multiple of the
// chunk rows M, strips aligned to chunks) and, as each row of w is produced,
// every column's interior elimination of its chunk (the data-dependent part of
// the y-chunk summary, see k_yreduce) is advanced; the running state lives in
// LDS.  At each chunk's interface row the planes E and Pf are written and the
// state restarts.
// LDS of one line group
template <typename T, int TR, bool FUSE>
struct XShared {
    T halo[2][2][TR];                        // segment edges of two rows: [row parity][first/last][seg]
    T tot[2][TR / 64][2];                    // wavefront scan totals: [fwd/bwd][wave][value]
    T y[FUSE ? 4 * kSeg * TR : 1];           // fused y-chunk state per column
};

// One strip (rows_per_strip rows from strip * rows_per_strip) of one line group.
// Every thread of the workgroup must call this with the same rows_per_strip
// (it synchronises the workgroup twice per row).
// STENCIL = false: the right-hand side of row j is rho_scale * (row j of A.u)
// instead of the 5-point assembly (line solves of a given field).
template <typename T, int TR, bool FUSE, bool STENCIL = true>
__device__ __forceinline__ void xsweep_strip(const XArgs<T>& A, const int strip, const int t,
                                             XShared<T, TR, FUSE>& sh)
{
    constexpr int E = kSeg;
    constexpr int NW = TR / 64;
    auto& s_halo = sh.halo;
    auto& s_tot = sh.tot;
    const int lane = t & 63;
    const int wv = t >> 6;
    const int nx = A.nx, ny = A.ny, nseg = A.nseg;
    const bool vec = A.vec != 0;
    const int RS = A.rows_per_strip;
    const int j0 = strip * RS;
    const int i0 = E * t;
    const bool act = t < nseg;
    const int L = act ? min(E, nx - i0) : 0;

    T um[E], uc[E], u1[E], u2[E];   // rows j-1, j, j+1, j+2 of u^n
    T rc[E], rn[E];                 // r of rows j, j+1
    T qc = T(0), qn = T(0);         // entry pivots of rows j, j+1

    auto load_u = [&](int row, T (&v)[E]) {
        if (act && row >= 0 && row < ny) load8<T>(A.u + (size_t)row * nx, i0, nx, vec, v);
        else {
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = T(0);
        }
    };
    auto load_rq = [&](int row, T (&v)[E], T& q) {
        if (act && row >= 0 && row < ny) {
            load8<T>(A.r + (size_t)row * nx, i0, nx, vec, v);
            q = A.qin[(size_t)row * nseg + t];
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = T(0);
            q = T(0);
        }
    };
    auto put_halo = [&](int row, const T (&v)[E]) {
        if (act) {
            T last = v[0];
#pragma unroll
            for (int e = 1; e < E; ++e)
                if (e == L - 1) last = v[e];
            s_halo[row & 1][0][t] = v[0];
            s_halo[row & 1][1][t] = last;
        }
    };

    T* ys = sh.y;
    auto ystate_reset = [&]() {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            ys[(0 * E + e) * TR + t] = T(0);   // q
            ys[(1 * E + e) * TR + t] = T(0);   // forward value
            ys[(2 * E + e) * TR + t] = T(1);   // running product of q
            ys[(3 * E + e) * TR + t] = T(0);   // first-value sum
        }
    };
    if constexpr (FUSE) ystate_reset();

    load_u(j0 - 1, um);
    load_u(j0, uc);
    load_u(j0 + 1, u1);
    load_rq(j0, rc, qc);
    put_halo(j0, uc);
    put_halo(j0 + 1, u1);
    __syncthreads();

    for (int it = 0; it < RS; ++it) {
        const int j = j0 + it;
        const bool live = j < ny;
        // prefetch
        load_u(live ? j + 2 : -1, u2);
        load_rq(live ? j + 1 : -1, rn, qn);

        // right-hand side of row j
        T rho[E];
        {
            const int p = j & 1;
            const T west0 = (act && t > 0) ? s_halo[p][1][t - 1] : T(0);
            const T eastL = (t + 1 < nseg) ? s_halo[p][0][t + 1] : T(0);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if constexpr (STENCIL) {
                    const T uw = (e == 0) ? west0 : uc[e - 1];
                    const T ue = (e == E - 1) ? eastL : uc[e + 1];
                    rho[e] = A.rho_scale * (T(2) * rc[e] * (((uw + ue) + (um[e] + u1[e])) - T(4) * uc[e]));
                } else {
                    rho[e] = A.rho_scale * uc[e];
                }
            }
        }
        if (live) {
            for (int q = 0; q < A.nsrc; ++q) {
                const int id = A.src_idx[q];
                if (id >= 0 && id / nx == j) {
                    const int i = id - j * nx - i0;
                    const T add = A.rho_scale * A.tau2 * A.src_amp[q];
#pragma unroll
                    for (int e = 0; e < E; ++e)
                        if (e == i) rho[e] += add;
                }
            }
        }

        // local elimination of the segment from its entry pivot
        T Ge[E], qe[E];
        T fG, fQ, H, Ev;
        {
            T q = qc, Gv = T(0), Qv = T(1), P = T(1), h = T(0), ee = T(0);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if (e < L) {
                    const T m = pivot_step<T>(rc[e], q);
                    Gv = fma_rn(m, rho[e], q * Gv);
                    Qv = q * Qv;
                    h = fma_rn(P, Gv, h);
                    ee = fma_rn(P, Qv, ee);
                    P = P * q;
                }
                Ge[e] = Gv;
                qe[e] = (e < L) ? q : T(0);
            }
            fG = Gv; fQ = Qv; H = h; Ev = ee;     // no node: identity (0, 1)
        }

        // forward scan across the line
        T gin;
        {
            T a = fG, b = fQ;
            wave_scan_fwd(a, b);
            if (lane == 63) { s_tot[0][wv][0] = a; s_tot[0][wv][1] = b; }
            const T xa = dpp<kWaveShr1>(T(0), a);
            const T xb = dpp<kWaveShr1>(T(1), b);
            __syncthreads();
            if (live && j + 2 < ny) put_halo(j + 2, u2);
            T carry = T(0);
            if constexpr (NW > 1) {
                T ta = (lane < NW) ? s_tot[0][lane < NW ? lane : 0][0] : T(0);
                T tb = (lane < NW) ? s_tot[0][lane < NW ? lane : 0][1] : T(1);
                compose_dpp<kRowShr + 1, 0xf>(ta, tb);
                compose_dpp<kRowShr + 2, 0xf>(ta, tb);
                compose_dpp<kRowShr + 4, 0xf>(ta, tb);
                compose_dpp<kRowShr + 8, 0xf>(ta, tb);
                carry = (wv > 0) ? readlane(ta, __builtin_amdgcn_readfirstlane(wv - 1)) : T(0);
            }
            gin = fma_rn(xb, carry, xa);
        }

        // backward scan across the line
        T dbelow;
        {
            T a = fma_rn(Ev, gin, H), b = fQ;
            if (!act) { a = T(0); b = T(1); }
            wave_scan_bwd(a, b, lane);
            if (lane == 0) { s_tot[1][wv][0] = a; s_tot[1][wv][1] = b; }
            const T ya = dpp<kWaveShl1>(T(0), a);
            const T yb = dpp<kWaveShl1>(T(1), b);
            __syncthreads();
            T carry = T(0);
            if constexpr (NW > 1) {
                T ta = (lane < NW) ? s_tot[1][lane < NW ? lane : 0][0] : T(0);
                T tb = (lane < NW) ? s_tot[1][lane < NW ? lane : 0][1] : T(1);
                compose_dpp<kRowShl + 1, 0xf>(ta, tb);
                compose_dpp<kRowShl + 2, 0xf>(ta, tb);
                compose_dpp<kRowShl + 4, 0xf>(ta, tb);
                compose_dpp<kRowShl + 8, 0xf>(ta, tb);
                carry = (wv + 1 < NW) ? readlane(ta, __builtin_amdgcn_readfirstlane(wv + 1)) : T(0);
            }
            dbelow = fma_rn(yb, carry, ya);
        }

        // back substitution, store
        T wout[E];
        {
            T x = dbelow, Q = T(1);
            T Qe[E];
#pragma unroll
            for (int e = 0; e < E; ++e) { Q = Q * qe[e]; Qe[e] = Q; }
#pragma unroll
            for (int e = E - 1; e >= 0; --e) {
                if (e < L) x = fma_rn(qe[e], x, fma_rn(Qe[e], gin, Ge[e]));
                wout[e] = x;
            }
            if (live && act) store8<T>(A.w + (size_t)j * nx, i0, nx, vec, wout);
        }

        if constexpr (FUSE) {
            const int c = j / A.M;
            const int kk = j - c * A.M;
            const int Lc = live ? min(A.M, ny - c * A.M) : 0;
            if (act && kk < Lc - 1) {
                // interior row of the y-chunk: advance every column's elimination
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    T q = ys[(0 * E + e) * TR + t];
                    T dv = ys[(1 * E + e) * TR + t];
                    T pi = ys[(2 * E + e) * TR + t];
                    T yp = ys[(3 * E + e) * TR + t];
                    const T m = pivot_step<T>(rc[e], q);
                    dv = fma_rn(rc[e], dv, wout[e]) * m;
                    yp = fma_rn(pi, dv, yp);
                    pi = pi * q;
                    ys[(0 * E + e) * TR + t] = q;
                    ys[(1 * E + e) * TR + t] = dv;
                    ys[(2 * E + e) * TR + t] = pi;
                    ys[(3 * E + e) * TR + t] = yp;
                }
            } else if (act && kk == Lc - 1) {
                // interface row of the chunk: E = wI + rI Pl and Pf, then restart
                const size_t pl = (size_t)A.K * A.nxp;
                const size_t o = ((size_t)(i0 / kPB) * A.K + c) * kPB + (i0 % kPB);
#pragma unroll
                for (int e = 0; e < E; ++e)
                    if (e < L) {
                        A.sum[4 * pl + o + e] = fma_rn(rc[e], ys[(1 * E + e) * TR + t], wout[e]);
                        A.sum[5 * pl + o + e] = ys[(3 * E + e) * TR + t];
                    }
                ystate_reset();
            }
        }

        qc = qn;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            um[e] = uc[e]; uc[e] = u1[e]; u1[e] = u2[e]; rc[e] = rn[e];
        }
    }
}

template <typename T, int TR, bool FUSE, bool STENCIL = true>
__global__ void __launch_bounds__(TR >= 256 ? TR : 256) k_xsweep(XArgs<T> A)
{
    constexpr int G = (TR >= 256 ? TR : 256) / TR;
    __shared__ XShared<T, TR, FUSE> sh[G];
    const int g = threadIdx.x / TR;
    xsweep_strip<T, TR, FUSE, STENCIL>(A, blockIdx.x * G + g, threadIdx.x - g * TR, sh[g]);
}

}  // namespace adw
