// fused4.hpp -- the one-pass FP32 step (the scheme and truncation bound of
// fused.hpp) on narrower tiles that keep r on chip: four nodes per lane, so a
// 240-wide tile still fills a wavefront with one x-row, and the LDS holds both
// w and r of the tile's 80 x-rows (2 x 80 x 240 floats), which the y-phase reads
// instead of reading r from memory a second time.  Included by adiwave.hip.
//
// A tile is Wt output columns (a multiple of 8, <= kF4Wmax) by 64 output rows.
//   Phase 1: x-lines of the 80 rows [r0 - 8, r0 + 72) on the column window
//            [c0 - 8, c0 + Wt + 8): one wavefront per row, four nodes per lane.
//            A lane's entry pivot is the full-line pivot of its 8-node segment
//            (odd lanes continue it over the four nodes of the lane before, whose
//            r they read across lanes); the elimination, the scans and the
//            back substitution are those of fused.hpp.  The Wt central values of
//            w and of r go to LDS.
//   Phase 2: y-lines: four windows of 32 rows per column, [r0 - 8 + 16 k,
//            r0 + 24 + 16 k), k = 0..3, one thread each, Thomas in registers on
//            w and r from LDS; the 16 central rows of d replace w.  Output rows
//            stay 9 rows from every cut, so the bound of fused.hpp holds as is.
//   Phase 3: u^{n+1} = 2 u^n - u^{n-1} + d, written over u^{n-1}, by the wavefront
//            that solved each x-row: u^n of the row is still in its registers
//            (not read again) and u^{n-1} was requested during the x-phase.

namespace adw {

constexpr int kF4Seg = 4;                      // nodes per lane
constexpr int kF4Wmax = 64 * kF4Seg - 2 * kFuKx;   // widest tile (240)
constexpr int kF4Hb = 16;                      // output rows per y-window
constexpr int kF4Nb = kF4Hb + 2 * kFuKy;       // rows of a y-window (32)
constexpr int kF4Win = kFuHt / kF4Hb;          // y-windows per column (4)

struct FShared4 {
    alignas(16) float w[kFuRows * kF4Wmax];
    alignas(16) float r[kFuRows * kF4Wmax];
    float src_add[kFuSrc];
    int src_pos[kFuSrc];   // (x-row << 16) | window column
    int src_n;             // -1: more than kFuSrc in this tile
};

__device__ __forceinline__ void fused4_tile(const FArgs& A, const int tile, FShared4& sh)
{
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int nx = A.nx, ny = A.ny, wt = A.wt;
    const int c0 = (tile % A.tiles_x) * wt;
    const int r0 = (tile / A.tiles_x) * kFuHt;
    const int nl = (wt + 2 * kFuKx) / kF4Seg;           // lanes of the x-window
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
            const bool hit = row >= 0 && xr >= 0 && xr < kFuRows && wc >= 0 && wc < nl * kF4Seg;
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

    constexpr int kR = kFuRows / 16;                           // consecutive x-rows per wavefront (5)
    const int xr0 = wv * kR;
    const int row_bytes = nx * 4;
    const int col0 = c0 - kFuKx + lane * kF4Seg;              // first column of the lane
    const int voff = lane < nl ? col0 * 4 : kFuOOB;
    float keep_u[kR][kF4Seg], keep_p[kR][kF4Seg];             // u^n and u^{n-1} of the wavefront's rows

    // ---------------------------------------------------------- phase 1: x
    {
        const bool inwin = lane < nl;
        const int seg = (c0 - kFuKx) / kSeg + (lane >> 1);     // its full-line 8-node segment
        const bool odd = lane & 1;
        const int qoff = inwin ? seg * 4 : kFuOOB;             // negative segments wrap past the row
        const int eoff = (lane == 0) ? (c0 - kFuKx - 1) * 4 : (lane == nl - 1) ? (c0 + wt + kFuKx) * 4 : kFuOOB;
        float ub[kR + 2][kF4Seg], eb[kR + 2], rb[kR][kF4Seg], qb[kR];
        auto row_ok = [&](int j) { return j >= 0 && j < ny; };
        auto load4 = [&](rsrc_t rs, float (&v)[kF4Seg]) {
            const f32x4 x = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, 0, 0));
            v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
        };
        auto load_u = [&](int j, float (&v)[kF4Seg], float& e) {
            const bool ok = row_ok(j);
            const rsrc_t rs = buf(A.uc + (size_t)(ok ? j : 0) * nx, ok ? row_bytes : 0);
            load4(rs, v);
            e = bload1<float>(rs, eoff);
        };
        auto load_r = [&](int j, float (&v)[kF4Seg], float& q) {
            const bool ok = row_ok(j);
            load4(buf(A.r + (size_t)(ok ? j : 0) * nx, ok ? row_bytes : 0), v);
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
            const float(&um)[kF4Seg] = ub[it];
            const float(&uc)[kF4Seg] = ub[it + 1];
            const float(&u1)[kF4Seg] = ub[it + 2];
            const float(&rc)[kF4Seg] = rb[it];
            const float eC = eb[it + 1];
            // u^n of the row stays for the update; u^{n-1} of the row is requested now,
            // for the tile's own nodes only (the halo nodes belong to other tiles)
#pragma unroll
            for (int e = 0; e < kF4Seg; ++e) keep_u[it][e] = uc[e];
            {
                const bool ok = row_ok(j);
                const bool own = xr >= kFuKy && xr < kFuKy + kFuHt && lane >= kFuKx / kF4Seg &&
                                 lane < nl - kFuKx / kF4Seg;
                const f32x4 pv = __builtin_bit_cast(
                    f32x4, __builtin_amdgcn_raw_buffer_load_b128(buf(A.up + (size_t)(ok ? j : 0) * nx, ok ? row_bytes : 0),
                                                                 own ? voff : kFuOOB, 0, kFuNT));
                keep_p[it][0] = pv.x; keep_p[it][1] = pv.y; keep_p[it][2] = pv.z; keep_p[it][3] = pv.w;
            }
            // right-hand side: west / east neighbours across lanes, window edges loaded
            float rho[kF4Seg];
            {
                const float west = dpp<kWaveShr1>(0.f, uc[kF4Seg - 1]);
                const float east = dpp<kWaveShl1>(0.f, uc[0]);
                const float w0 = lane == 0 ? eC : west;
                const float eL = lane == nl - 1 ? eC : east;
#pragma unroll
                for (int e = 0; e < kF4Seg; ++e) {
                    const float uw = e == 0 ? w0 : uc[e - 1];
                    const float ue = e == kF4Seg - 1 ? eL : uc[e + 1];
                    rho[e] = 2.f * (rc[e] * (((uw + ue) + (um[e] + u1[e])) - 4.f * uc[e]));
                }
            }
            if (ns > 0) {
                for (int s = 0; s < ns; ++s) {
                    const int pos = sh.src_pos[s];
                    if ((pos >> 16) == xr) {
                        const int i = (pos & 0xffff) - lane * kF4Seg;
                        const float add = sh.src_add[s];
#pragma unroll
                        for (int e = 0; e < kF4Seg; ++e)
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
                        for (int e = 0; e < kF4Seg; ++e)
                            if (e == i && inwin) rho[e] += add;
                    }
                }
            }
            // entry pivot: the segment's full-line pivot, carried by odd lanes over
            // the four nodes of the even lane before them (same arithmetic as the
            // elimination, so the pivots are those of the full line)
            float q = qb[it];
            {
                float qo = q;
#pragma unroll
                for (int e = 0; e < kF4Seg; ++e) (void)pivot_step<float>(dpp<kRowShr + 1>(0.f, rc[e]), qo);
                q = odd ? qo : q;
            }
            // lane elimination from the entry pivot (zero rows decouple)
            float Ge[kF4Seg], qe[kF4Seg], Qe[kF4Seg];
            float fG, fQ, H, Ev;
            {
                float Gv = 0.f, Qv = 1.f, h = 0.f, ee = 0.f;
#pragma unroll
                for (int e = 0; e < kF4Seg; ++e) {
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
            float wout[kF4Seg];
            {
                float x = dbelow;
#pragma unroll
                for (int e = kF4Seg - 1; e >= 0; --e) {
                    x = fma_rn(qe[e], x, fma_rn(Qe[e], gin, Ge[e]));
                    wout[e] = x;
                }
            }
            // central columns of w and r to LDS (lanes 2 .. nl-3 hold columns c0 .. c0+wt-1)
            if (lane >= kFuKx / kF4Seg && lane < nl - kFuKx / kF4Seg) {
                // in float4 units (wt is a multiple of 8): one 16-byte LDS write per lane
                const int o4 = xr * (wt / 4) + (lane - kFuKx / kF4Seg);
                reinterpret_cast<float4*>(sh.w)[o4] = make_float4(wout[0], wout[1], wout[2], wout[3]);
                reinterpret_cast<float4*>(sh.r)[o4] = make_float4(rc[0], rc[1], rc[2], rc[3]);
            }
        }
    }
    __syncthreads();

    // ------------------------------------------------- phase 2: y windows
    const bool ythr = t < kF4Win * wt;
    const int win = ythr ? t / wt : 0;
    const int ci = ythr ? t - win * wt : 0;
    float gk[kF4Nb], qk[kF4Nb];
    if (ythr) {
        float q = 0.f, g = 0.f;
        int o = (kF4Hb * win) * wt + ci;                     // LDS index of (window row k, ci)
#pragma unroll
        for (int k = 0; k < kF4Nb; ++k, o += wt) {
            const float m = pivot_step<float>(sh.r[o], q);
            g = fma_rn(m, sh.w[o], q * g);
            gk[k] = g;
            qk[k] = q;
        }
    }
    __syncthreads();
    if (ythr) {
        float d = 0.f;
        float* dcol = sh.w + (kF4Hb * win) * wt + ci;
#pragma unroll
        for (int k = kF4Nb - 1; k >= kFuKy; --k) {
            d = fma_rn(qk[k], d, gk[k]);
            if (k < kFuKy + kF4Hb) dcol[k * wt] = d;
        }
    }

    // ------------------------------------------------------ phase 3: update
    __syncthreads();
    {
        const bool outlane = lane >= kFuKx / kF4Seg && lane < nl - kFuKx / kF4Seg;
#pragma unroll
        for (int it = 0; it < kR; ++it) {
            const int xr = xr0 + it;
            const int j = r0 - kFuKy + xr;
            if (xr >= kFuKy && xr < kFuKy + kFuHt && outlane) {
                const float4 dv = reinterpret_cast<const float4*>(sh.w)[xr * (wt / 4) + (lane - kFuKx / kF4Seg)];
                const f32x4 o = {fma_rn(2.f, keep_u[it][0], -keep_p[it][0]) + dv.x,
                                 fma_rn(2.f, keep_u[it][1], -keep_p[it][1]) + dv.y,
                                 fma_rn(2.f, keep_u[it][2], -keep_p[it][2]) + dv.z,
                                 fma_rn(2.f, keep_u[it][3], -keep_p[it][3]) + dv.w};
                const bool ok = j >= 0 && j < ny;
                __builtin_amdgcn_raw_buffer_store_b128(
                    __builtin_bit_cast(i32x4, o), buf(static_cast<const float*>(A.up) + (size_t)(ok ? j : 0) * nx, ok ? row_bytes : 0),
                    voff, 0, kFuNT);
            }
        }
    }
}

__global__ void __launch_bounds__(1024) k_fused4(FArgs A)
{
    __shared__ FShared4 sh;
    rec_tap<float>(A.uc, A.rec_idx, A.rec_out, A.nrec, (long long)A.nx * A.ny);
    const int tile = A.xcd_map ? xcd_band(blockIdx.x) : (int)blockIdx.x;
    if (tile >= A.tiles) return;
    fused4_tile(A, tile, sh);
}

}  // namespace adw
