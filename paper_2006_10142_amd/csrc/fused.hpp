// fused.hpp -- the whole ADI step in one pass (FP32): right-hand side, x-lines,
// y-lines and the update of each output tile from u^n, u^{n-1} and r, without
// writing the x-sweep result to memory.  Included by adiwave.hip.
//
// Truncated line solves.  Every line system -r x_{i-1} + (1 + 2r) x_i - r x_{i+1}
// = b is strictly diagonally dominant, and all its elimination pivots q lie in
// [0, qs], qs = (1 + 2 rm - sqrt(1 + 4 rm)) / (2 rm) the fixed point of the pivot
// map at the largest coefficient rm.  Solving the line on a window whose carries
// are set to zero at its ends (x-lines: the full-line elimination with the
// forward carry entering the window and the back-substitution value leaving it
// replaced by 0; y-lines: the window's own system with zero values beyond it)
// changes the solution at distance d from a cut by at most qs^d max|x|: the
// dropped carry is multiplied by one pivot per node it crosses.  Output nodes are
// 9 columns from the x-cuts and 9 rows from the y-cuts, and the y-solve does not
// amplify errors of its right-hand side in the max norm (its inverse has norm
// <= 1), so one step differs from the exact two-pass step by at most
//     2 qs^9 max|w| + 2 qs^9 max|d|  <=  4 qs^9 max|w|,
// which the host keeps below 2^-24 (half an FP32 ulp) by enabling this path only
// when rm is small enough (rm <= 0.18); otherwise the exact path runs.
//
// A tile is Wt output columns (a multiple of 8, <= 496) by 64 output rows.
//   Phase 1: x-lines of the 80 rows [r0 - 8, r0 + 72), each on the column window
//            [c0 - 8, c0 + Wt + 8): one wavefront per row, 8 nodes per lane, the
//            segment scheme of xsweep.hpp with the full-line entry pivots; the Wt
//            central values of w go to LDS (80 x Wt).
//   Phase 2: y-lines: two windows of 48 rows per column ([r0 - 8, r0 + 40) and
//            [r0 + 24, r0 + 72)), one thread each, Thomas in registers; the 32
//            central rows of d replace w in LDS.
//   Phase 3: u^{n+1} = 2 u^n - u^{n-1} + d over the tile, written over u^{n-1}
//            (each node of u^{n-1} is read only by the tile that owns it).
// Rows and columns outside the grid read as zero through the buffer range checks:
// such nodes have r = 0 and decouple, which is the zero Dirichlet boundary.

namespace adw {

constexpr int kFuKx = 8;            // x-halo columns on each side (one 8-node segment)
constexpr int kFuKy = 8;            // y-halo rows on each side
constexpr int kFuHb = 32;           // output rows per y-window
constexpr int kFuNb = kFuHb + 2 * kFuKy;   // rows of a y-window (48)
constexpr int kFuHt = 2 * kFuHb;    // output rows per tile (64)
constexpr int kFuRows = kFuHt + 2 * kFuKy;   // x-rows per tile (80)
constexpr int kFuWmax = 64 * kSeg - 2 * kFuKx;   // widest tile (496)
constexpr int kFuSrc = 32;          // point sources staged per tile
constexpr int kFuRing = 16;         // rows of r requested ahead in a y-window
constexpr int kFuUp = (kFuHt * kFuWmax / 4 + 1023) / 1024;   // float4 updated per thread (8)
constexpr int kFuNT = 2;            // buffer cache policy: non-temporal (a last use of the line)
constexpr int kFuOOB = 0x40000000;  // byte offset beyond every buffer range used here
                                    // (grids hold at most 2^27 values, 2^29 bytes)

template <typename T>
struct FArgsT {
    const T* uc;         // u^n
    T* up;               // u^{n-1} in, u^{n+1} out
    const T* r;
    const T* qin;        // full-line entry pivot of every 8-node x-segment
    int nx, ny, nseg;
    int wt;              // output columns per tile (multiple of 8)
    int tiles_x, tiles;  // tiles across, total tiles
    int wide;            // column strips (fusedr.hpp): strips 0..wide-1 are wt wide, the others wt - 8
    int xcd_map;         // 1: block -> tile map that keeps neighbours on one XCD
    int hs;              // column strips (fusedr.hpp): output rows per strip segment
    T tau2;
    int nsrc;
    const int* src_idx;
    const T* src_amp;
    int nrec;            // receivers of the previous step, sampled from uc (see rec_tap)
    const int* rec_idx;
    T* rec_out;
};
using FArgs = FArgsT<float>;   // the tile kernels are FP32; the column strips take both

struct FShared {
    float w[kFuRows * kFuWmax];
    float src_add[kFuSrc];
    int src_pos[kFuSrc];   // (x-row << 16) | window column
    int src_n;             // -1: more than kFuSrc in this tile
};

// inclusive suffix (lanes l..63) of two-component affine maps over the wavefront
__device__ __forceinline__ void wave_scan_bwd2(float& a, float& b, int lane)
{
    fu_row_scan_bwd(a, b);
    const float a16 = readlane(a, 16), b16 = readlane(b, 16);
    const float a32 = readlane(a, 32), b32 = readlane(b, 32);
    const float a48 = readlane(a, 48), b48 = readlane(b, 48);
    const float a23 = fma_rn(b32, a48, a32), b23 = b32 * b48;
    const float a13 = fma_rn(b16, a23, a16), b13 = b16 * b23;
    float ca = 0.f, cb = 1.f;
    if (lane < 16) { ca = a13; cb = b13; }
    else if (lane < 32) { ca = a23; cb = b23; }
    else if (lane < 48) { ca = a48; cb = b48; }
    a = fma_rn(b, ca, a);
    b = b * cb;
}

// one value through a buffer resource, marked as the last use of its line (the
// x-phase read it first; the line should not displace data still to be re-read)
__device__ __forceinline__ float fu_load1_nt(rsrc_t rs, int voff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, 0, kFuNT));
}

// block -> work index: the blocks of one XCD (b mod 8) take one contiguous band
// of indices, so tiles that share halo rows share an L2 (gridDim.x is a
// multiple of 8)
__device__ __forceinline__ int xcd_band(int b) { return (b & 7) * (int)(gridDim.x >> 3) + (b >> 3); }

// one tile of one grid; every thread of the 1024-thread workgroup takes part
__device__ __forceinline__ void fused_tile(const FArgs& A, const int tile, FShared& sh)
{
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int nx = A.nx, ny = A.ny, wt = A.wt;
    const int c0 = (tile % A.tiles_x) * wt;
    const int r0 = (tile / A.tiles_x) * kFuHt;
    const int nl = (wt + 2 * kFuKx) / kSeg;             // lanes of the x-window
    const long long npts = (long long)nx * ny;

    // ---- point sources of the tile's x-rows and x-window, in source order
    if (t < 64) {
        int n = 0;
        for (int base = 0; base < A.nsrc; base += 64) {
            const int qq = base + t;
            int id = -1;
            float amp = 0.f;
            if (qq < A.nsrc) { id = A.src_idx[qq]; amp = A.src_amp[qq]; }
            const int row = (id >= 0 && id < npts) ? id / nx : -1;
            const int col = row >= 0 ? id - row * nx : 0;
            const int xr = row - (r0 - kFuKy);
            const int wc = col - (c0 - kFuKx);
            const bool hit = row >= 0 && xr >= 0 && xr < kFuRows && wc >= 0 && wc < nl * kSeg;
            const unsigned long long mask = __ballot(hit);
            const int before = __popcll(mask & ((1ull << t) - 1ull));
            if (hit && n + before < kFuSrc) {
                sh.src_add[n + before] = A.tau2 * amp;
                sh.src_pos[n + before] = (xr << 16) | wc;
            }
            n += __popcll(mask);
        }
        if (t == 0) sh.src_n = n <= kFuSrc ? n : -1;
    }
    __syncthreads();

    // ---------------------------------------------------------- phase 1: x
    {
        const bool inwin = lane < nl;
        const int seg = (c0 - kFuKx) / kSeg + lane;        // full-line segment index
        const int col0 = seg * kSeg;
        const int voff = inwin ? col0 * 4 : kFuOOB;
        const int qoff = inwin ? seg * 4 : kFuOOB;           // negative segments wrap past the row
        const int eoff = (lane == 0) ? (c0 - kFuKx - 1) * 4 : (lane == nl - 1) ? (c0 + wt + kFuKx) * 4 : kFuOOB;
        const int row_bytes = nx * 4;
        constexpr int kR = kFuRows / 16;                    // consecutive x-rows per wavefront (5)
        const int xr0 = wv * kR;
        // rows of u^n j0-1 .. j0+kR and of r j0 .. j0+kR-1, each requested two rows
        // before the row that first needs it
        float ub[kR + 2][kSeg], eb[kR + 2], rb[kR][kSeg], qb[kR];
        auto row_ok = [&](int j) { return j >= 0 && j < ny; };
        auto load_u = [&](int j, float (&v)[kSeg], float& e) {
            const bool ok = row_ok(j);
            const rsrc_t rs = buf(A.uc + (size_t)(ok ? j : 0) * nx, ok ? row_bytes : 0);
            bload8<float>(rs, voff, v);
            e = bload1<float>(rs, eoff);
        };
        auto load_r = [&](int j, float (&v)[kSeg], float& q) {
            const bool ok = row_ok(j);
            bload8<float>(buf(A.r + (size_t)(ok ? j : 0) * nx, ok ? row_bytes : 0), voff, v);
            q = bload1<float>(buf(A.qin + (size_t)(ok ? j : 0) * A.nseg, ok ? A.nseg * 4 : 0), qoff);
        };
        const int j0 = r0 - kFuKy + xr0;
#pragma unroll
        for (int k = 0; k < 4; ++k) load_u(j0 - 1 + k, ub[k], eb[k]);
        load_r(j0, rb[0], qb[0]);
        load_r(j0 + 1, rb[1], qb[1]);
        const int ns = sh.src_n;
#pragma unroll
        for (int it = 0; it < kR; ++it) {
            const int xr = xr0 + it;
            const int j = j0 + it;
            if (it + 4 < kR + 2) load_u(j + 3, ub[it + 4], eb[it + 4]);
            if (it + 2 < kR) load_r(j + 2, rb[it + 2], qb[it + 2]);
            const float(&um)[kSeg] = ub[it];
            const float(&uc)[kSeg] = ub[it + 1];
            const float(&u1)[kSeg] = ub[it + 2];
            const float(&rc)[kSeg] = rb[it];
            const float eC = eb[it + 1], qc = qb[it];
            // right-hand side: west / east neighbours across lanes, window edges loaded
            float rho[kSeg];
            {
                const float west = dpp<kWaveShr1>(0.f, uc[kSeg - 1]);
                const float east = dpp<kWaveShl1>(0.f, uc[0]);
                const float w0 = lane == 0 ? eC : west;
                const float eL = lane == nl - 1 ? eC : east;
#pragma unroll
                for (int e = 0; e < kSeg; ++e) {
                    const float uw = e == 0 ? w0 : uc[e - 1];
                    const float ue = e == kSeg - 1 ? eL : uc[e + 1];
                    rho[e] = 2.f * (rc[e] * (((uw + ue) + (um[e] + u1[e])) - 4.f * uc[e]));
                }
            }
            if (ns > 0) {
                for (int s = 0; s < ns; ++s) {
                    const int pos = sh.src_pos[s];
                    if ((pos >> 16) == xr) {
                        const int i = (pos & 0xffff) - lane * kSeg;
                        const float add = sh.src_add[s];
#pragma unroll
                        for (int e = 0; e < kSeg; ++e)
                            if (e == i) rho[e] += add;
                    }
                }
            } else if (ns < 0 && row_ok(j)) {
                for (int s = 0; s < A.nsrc; ++s) {
                    const int id = A.src_idx[s];
                    if (id >= 0 && id < npts && id / nx == j) {
                        const int i = id - j * nx - col0;
                        const float add = A.tau2 * A.src_amp[s];
#pragma unroll
                        for (int e = 0; e < kSeg; ++e)
                            if (e == i && inwin) rho[e] += add;
                    }
                }
            }
            // segment elimination from the full-line entry pivot (zero rows decouple)
            float Ge[kSeg], qe[kSeg], Qe[kSeg];
            float fG, fQ, H, Ev;
            {
                float q = qc, Gv = 0.f, Qv = 1.f, h = 0.f, ee = 0.f;
#pragma unroll
                for (int e = 0; e < kSeg; ++e) {
                    const float m = pivot_step<float>(rc[e], q);
                    const float P = Qv;
                    Gv = fma_rn(m, rho[e], q * Gv);
                    Qv = q * Qv;
                    h = fma_rn(P, Gv, h);
                    ee = fma_rn(P, Qv, ee);
                    Ge[e] = Gv;
                    qe[e] = q;
                    Qe[e] = Qv;
                }
                fG = Gv; fQ = Qv; H = h; Ev = ee;
            }
            // forward carries within the window (zero entering lane 0)
            float a = fG, b = fQ;
            fu_scan_fwd(a, b);
            const float gin = dpp<kWaveShr1>(0.f, a);
            // backward values within the window (zero leaving the last lane)
            float ba = inwin ? fma_rn(Ev, gin, H) : 0.f, bb = inwin ? fQ : 1.f;
            wave_scan_bwd2(ba, bb, lane);
            const float dbelow = dpp<kWaveShl1>(0.f, ba);
            float wout[kSeg];
            {
                float x = dbelow;
#pragma unroll
                for (int e = kSeg - 1; e >= 0; --e) {
                    x = fma_rn(qe[e], x, fma_rn(Qe[e], gin, Ge[e]));
                    wout[e] = x;
                }
            }
            // central columns to LDS (lanes 1 .. nl-2 hold columns c0 .. c0+wt-1)
            if (lane >= kFuKx / kSeg && lane < nl - kFuKx / kSeg) {
                float* dst = sh.w + xr * wt + (lane - kFuKx / kSeg) * kSeg;
                *reinterpret_cast<float4*>(dst) = make_float4(wout[0], wout[1], wout[2], wout[3]);
                *reinterpret_cast<float4*>(dst + 4) = make_float4(wout[4], wout[5], wout[6], wout[7]);
            }
        }
    }

    // ------------------------------------------------- phase 2: y windows
    const bool ythr = t < 2 * wt;
    const int ci = ythr ? (t < wt ? t : t - wt) : 0;
    const int half = t < wt ? 0 : 1;
    const int gcol = c0 + ci;
    const int jtop = r0 - kFuKy + kFuHb * half;             // global row of window row 0
    const rsrc_t rall = buf(A.r, (int)(npts * 4));
    // byte offset of node (jtop + k, gcol) is off + k * rowb, in 32-bit unsigned
    // arithmetic: rows above the grid wrap to offsets near 2^32 and rows below it
    // lie past the end, both outside the buffer range (they read as zero); columns
    // past the grid start at 2^31 and stay outside it
    const unsigned rowb = (unsigned)nx * 4u;
    unsigned off = gcol < nx ? (unsigned)(jtop * nx + gcol) * 4u : 0x80000000u;
    // r of the window, kFuRing rows ahead; the first rows are requested before the
    // barrier that ends the x-phase (a barrier waits for LDS traffic only)
    float rbuf[kFuRing];
    if (ythr) {
#pragma unroll
        for (int k = 0; k < kFuRing; ++k, off += rowb) rbuf[k] = fu_load1_nt(rall, (int)off);
    }
    __syncthreads();
    float gk[kFuNb], qk[kFuNb];
    if (ythr) {
        float q = 0.f, g = 0.f;
        int wo = (kFuHb * half) * wt + ci;                 // LDS index of (window row k, ci)
#pragma unroll
        for (int k = 0; k < kFuNb; ++k, wo += wt) {
            const float rk = rbuf[k % kFuRing];
            if (k + kFuRing < kFuNb) {
                rbuf[k % kFuRing] = fu_load1_nt(rall, (int)off);
                off += rowb;
            }
            const float m = pivot_step<float>(rk, q);
            g = fma_rn(m, sh.w[wo], q * g);
            gk[k] = g;
            qk[k] = q;
        }
    }
    __syncthreads();
    if (ythr) {
        float d = 0.f;
        float* dcol = sh.w + (kFuHb * half) * wt + ci;
#pragma unroll
        for (int k = kFuNb - 1; k >= 0; --k) {
            d = fma_rn(qk[k], d, gk[k]);
            if (k >= kFuKy && k < kFuKy + kFuHb) dcol[k * wt] = d;
        }
    }

    // ------------------------------------------------------ phase 3: update
    // every float4 of the tile's u^n and u^{n-1} that this thread updates is
    // requested before the barrier, all at once; these loads and the stores of
    // u^{n+1} are last uses of their lines within the step (non-temporal), so
    // they leave L2 room for the rows that later tiles and phases re-read
    const int nq = wt / 4;                                  // float4 per tile row
    const int total = kFuHt * nq;
    const int lim = (int)(npts * 4);
    const rsrc_t ruc = buf(A.uc, lim);
    const rsrc_t rup = buf(static_cast<const float*>(A.up), lim);
    f32x4 cv[kFuUp], pv[kFuUp];
    int uoff[kFuUp];
#pragma unroll
    for (int s = 0; s < kFuUp; ++s) {
        const int idx = s * 1024 + t;
        const int orow = idx / nq, oq = idx - orow * nq;
        const int j = r0 + orow, i = c0 + 4 * oq;
        uoff[s] = (idx < total && j < ny && i < nx) ? (j * nx + i) * 4 : kFuOOB;
        cv[s] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(ruc, uoff[s], 0, kFuNT));
        pv[s] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rup, uoff[s], 0, kFuNT));
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kFuUp; ++s) {
        const int idx = s * 1024 + t;
        if (idx < total) {
            const int orow = idx / nq, oq = idx - orow * nq;
            const float4 dv = *reinterpret_cast<const float4*>(sh.w + (kFuKy + orow) * wt + 4 * oq);
            const f32x4 o = {fma_rn(2.f, cv[s].x, -pv[s].x) + dv.x, fma_rn(2.f, cv[s].y, -pv[s].y) + dv.y,
                             fma_rn(2.f, cv[s].z, -pv[s].z) + dv.z, fma_rn(2.f, cv[s].w, -pv[s].w) + dv.w};
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(i32x4, o), rup, uoff[s], 0, kFuNT);
        }
    }
}

__global__ void __launch_bounds__(1024) k_fused(FArgs A)
{
    __shared__ FShared sh;
    rec_tap<float>(A.uc, A.rec_idx, A.rec_out, A.nrec, (long long)A.nx * A.ny);
    const int tile = A.xcd_map ? xcd_band(blockIdx.x) : (int)blockIdx.x;
    if (tile >= A.tiles) return;
    fused_tile(A, tile, sh);
}

}  // namespace adw

namespace adw {

// largest r (r >= 0, so the float bits order like the values): per-block
// maximum, then one atomic per block on the bit pattern
__global__ void __launch_bounds__(256) k_rmax(const float* __restrict__ r, long long n, unsigned int* out)
{
    __shared__ float red[256];
    float m = 0.f;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        m = fmaxf(m, r[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, __float_as_uint(red[0]));
}

// the same for FP64 r (the double bits order like the values)
__global__ void __launch_bounds__(256) k_rmax64(const double* __restrict__ r, long long n, unsigned long long* out)
{
    __shared__ double red[256];
    double m = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        m = fmax(m, r[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(red[0]));
}

}  // namespace adw
