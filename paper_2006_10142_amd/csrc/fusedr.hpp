// fusedr.hpp -- the one-pass step (FP32) on column strips with the work split by
// role, so that the y-lines run while the next x-rows are solved and loaded.
// Included by adiwave.hip after fused4.hpp, whose x-row scheme it uses.
//
// A workgroup owns a strip of Wt output columns (a multiple of 8, <= 240; the plan
// mixes two widths 8 apart so that the strips cover the grid evenly) and hs
// output rows, and walks down it in bands of 24 x-rows; band k holds the x-rows
// [r0 - 8 + 24k, r0 + 16 + 24k).
//   x-role (12 wavefronts): two x-rows each per band, four nodes per lane, on
//     the window [c0 - 8, c0 + Wt + 8) as fused4.hpp, except for the entry pivots
//     (below); w, r and u^n of the central columns go to rings of 56 rows in LDS.
//     The inputs of band k + 1 are in registers, and those of band k + 2 are
//     requested as soon as band k is solved.
//   Entry pivots: each lane rebuilds the elimination pivot entering its four
//     nodes by running the pivot map q -> r / (1 + r (2 - q)) from q = 0 over the
//     six nodes before them, instead of reading the full-line value.  The map
//     contracts by its derivative q^2 <= qs^2 (qs < 0.14 for r <= 0.18), so after
//     six nodes the start value is forgotten to a factor below 1e-11: the pivot is
//     the full-line one up to rounding.  The window's first two lanes have fewer
//     nodes before them inside the window and start from zero at its edge: that is
//     the window's own system, the same truncation as the y-lines', covered by the
//     bound of fused.hpp (the cut is 9 columns from the first output column).
//   y-role (4 wavefronts, one thread per column): in the same pass, band k - 1.
//     The forward elimination of each y-line continues down the strip from row
//     r0 - 8 (zero carries: the upper cut, 9 rows above the first output row),
//     over the band's 24 rows (g and the pivots replace w and r in the ring).  The back
//     substitution starts at the band's last row with a zero value (the lower
//     cut, 9 rows below the band's last output row), runs up through the band
//     and through the 8 look-ahead rows kept in the ring by the band before, and
//     updates the output rows [r0 - 16 + 24k, r0 + 8 + 24k) (band 0: [r0, r0 + 8))
//     as it goes: u^{n+1} = 2 u^n - u^{n-1} + d, with u^n from its ring (the
//     x-role had it in registers) and u^{n-1} requested a pass ahead.  The
//     band's last 8 rows (g, pivots and u^n) stay in the rings.
// Each output row is the solution of a y-window whose cuts are at least 9 rows
// away, and each x-row that of an x-window cut 9 columns away, so the truncation
// bound of fused.hpp holds unchanged.  A barrier separates the passes: the
// ring's 56 rows hold the band being solved (24), the band being eliminated (24)
// and the look-ahead rows before it (8), and these never overlap.

namespace adw {

constexpr int kFrB = 24;                   // x-rows per band
constexpr int kFrR = 2 * kFrB + kFuKy;     // ring rows (56)
constexpr int kFrY = 4;                    // y-role wavefronts (one thread per column)
constexpr int kFrX = 12;                   // x-role wavefronts (8, with three x-rows each, measured slower)
constexpr int kFrXr = kFrB / kFrX;         // x-rows per x-role wavefront per band (2)
constexpr int kFrThreads = 64 * (kFrY + kFrX);   // workgroup size (1024: at most 128 VGPRs a thread)
static_assert(kFrB % kFrX == 0, "every x-role wavefront takes the same number of x-rows");
constexpr int kFrS = kF4Wmax;              // ring row stride (240)
constexpr int kFrHmin = 256;               // shortest strip segment the plan picks by itself

struct FRShared {
    alignas(16) float w[kFrR * kFrS];   // w of the x-rows, then g once the y-role has eliminated them
    alignas(16) float r[kFrR * kFrS];   // r of the x-rows, then the y-lines' pivots
    alignas(16) float u[kFrR * kFrS];   // u^n of the x-rows, read again by the update
    float src_add[kFuSrc];
    int src_row[kFuSrc];
    int src_wc[kFuSrc];
    int src_n;              // -1: more than kFuSrc in this strip
};

static_assert(sizeof(FRShared) <= 160 * 1024, "the strip ring exceeds the LDS of a workgroup");

// x-role inputs of one band: u^n rows j-1 .. j+kFrXr and r rows j .. j+kFrXr-1
// of the wavefront's x-rows, with the window-edge values
struct FRIn {
    float u[kFrXr + 2][kF4Seg];
    float e[kFrXr + 2];
    float r[kFrXr][kF4Seg];
};

__global__ void __launch_bounds__(kFrThreads) k_fusedr(FArgs A)
{
    __shared__ FRShared sh;
    rec_tap<float>(A.uc, A.rec_idx, A.rec_out, A.nrec, (long long)A.nx * A.ny);
    // neighbouring strips of a segment row run on one XCD (their halo columns meet
    // in that XCD's L2): the grid is a multiple of 8 and blocks past the tiles exit
    const int blk = A.xcd_map ? xcd_band(blockIdx.x) : (int)blockIdx.x;
    if (blk >= A.tiles) return;
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int nx = A.nx, ny = A.ny;
    const int sx = blk % A.tiles_x;                       // strip index: the first A.wide are
    const int wt = sx < A.wide ? A.wt : A.wt - 8;         // A.wt wide, the others 8 narrower
    const int c0 = sx * A.wt - (sx > A.wide ? (sx - A.wide) * 8 : 0);
    const int r0 = (blk / A.tiles_x) * A.hs;
    const int r1 = min(r0 + A.hs, ny);
    const int nb = r1 - r0 <= kFuKy ? 1 : 1 + (r1 - r0 - kFuKy + kFrB - 1) / kFrB;
    const int nl = (wt + 2 * kFuKx) / kF4Seg;            // lanes of the x-window
    const long long npts = (long long)nx * ny;
    const int xr_lo = r0 - kFuKy, xr_hi = xr_lo + kFrB * nb;   // x-rows of the strip
    // ring slot of x-row xr_lo + 24 k + i (0 <= i < 56): the band's first slot
    // (24 k mod 56) is carried from band to band, so no division is needed
    auto wrap = [](int s) { return s >= kFrR ? s - kFrR : s; };
    auto next_base = [&](int sb) { return wrap(sb + kFrB); };

    // ---- point sources of the strip's x-rows and x-window, in source order
    if (t < 64) {
        int n = 0;
        for (int base = 0; base < A.nsrc; base += 64) {
            const int qq = base + t;
            int id = -1;
            float amp = 0.f;
            if (qq < A.nsrc) { id = A.src_idx[qq]; amp = A.src_amp[qq]; }
            const int row = (id >= 0 && id < npts) ? id / nx : -1;
            const int col = row >= 0 ? id - row * nx : 0;
            const int wc = col - (c0 - kFuKx);
            const bool hit = row >= 0 && row >= xr_lo && row < xr_hi && wc >= 0 && wc < nl * kF4Seg;
            const unsigned long long mask = __ballot(hit);
            const int before = __popcll(mask & ((1ull << t) - 1ull));
            if (hit && n + before < kFuSrc) {
                sh.src_add[n + before] = A.tau2 * amp;
                sh.src_row[n + before] = row;
                sh.src_wc[n + before] = wc;
            }
            n += __popcll(mask);
        }
        if (t == 0) sh.src_n = n <= kFuSrc ? n : -1;
    }
    __syncthreads();
    const int ns = sh.src_n;
    const int row_bytes = nx * 4;
    auto row_ok = [&](int j) { return j >= 0 && j < ny; };

    // ---- x-role constants
    const int xw = wv - kFrY;                               // x-role wavefront index
    const bool inwin = lane < nl;
    const int col0 = c0 - kFuKx + lane * kF4Seg;            // first column of the lane
    // One buffer resource per plane: a row is reached through the scalar offset, and
    // whatever lies outside the grid (the lanes or edge values past a wall, whole rows
    // above or below it, the bands past the strip's last) through a vector offset past
    // every range, which the range check turns into zeros without a memory access.
    const int ecol = (lane == 0) ? c0 - kFuKx - 1 : (lane == nl - 1) ? c0 + wt + kFuKx : -1;
    const int voff = (inwin && col0 >= 0 && col0 < nx) ? col0 * 4 : kFuOOB;
    const int eoff = (ecol >= 0 && ecol < nx) ? ecol * 4 : kFuOOB;
    const int plane = (int)(npts * 4);
    const rsrc_t ru_all = buf(A.uc, plane);
    const rsrc_t rr_all = buf(A.r, plane);
    auto load4 = [&](rsrc_t rs, int vo, int so, float (&v)[kF4Seg]) {
        const f32x4 x = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, vo, so, 0));
        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    };
    auto load1 = [&](rsrc_t rs, int vo, int so) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, vo, so, 0));
    };
    // pieces of band k's inputs: u^n row j-1+i (with its window-edge values), and
    // r row j+i with its entry pivots, j = the wavefront's first x-row of band k
    auto load_u = [&](int k, int i, FRIn& P) {
        const int jj = xr_lo + kFrB * k + kFrXr * xw - 1 + i;
        const bool ok = row_ok(jj) && k < nb;
        const int so = ok ? jj * row_bytes : 0;
        load4(ru_all, ok ? voff : kFuOOB, so, P.u[i]);
        P.e[i] = load1(ru_all, ok ? eoff : kFuOOB, so);
    };
    auto load_r = [&](int k, int i, FRIn& P) {
        const int jj = xr_lo + kFrB * k + kFrXr * xw + i;
        const bool ok = row_ok(jj) && k < nb;
        load4(rr_all, ok ? voff : kFuOOB, ok ? jj * row_bytes : 0, P.r[i]);
    };
    auto load_band = [&](int k, FRIn& P) {
#pragma unroll
        for (int i = 0; i < kFrXr + 2; ++i) load_u(k, i, P);
#pragma unroll
        for (int i = 0; i < kFrXr; ++i) load_r(k, i, P);
    };
    // the x-rows of band k from P (sb: the band's first ring slot); w and r of the
    // central columns to the ring
    auto x_band = [&](int k, int sb, const FRIn& P) {
#pragma unroll
        for (int it = 0; it < kFrXr; ++it) {
            const int j = xr_lo + kFrB * k + kFrXr * xw + it;
            const float(&um)[kF4Seg] = P.u[it];
            const float(&uc)[kF4Seg] = P.u[it + 1];
            const float(&u1)[kF4Seg] = P.u[it + 2];
            const float(&rc)[kF4Seg] = P.r[it];
            const float eC = P.e[it + 1];
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
                    if (sh.src_row[s] == j) {
                        const int i = sh.src_wc[s] - lane * kF4Seg;
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
            // entry pivot of the lane, rebuilt from zero over the six nodes before it
            // (see the header: within rounding of the full-line pivot; at the window's
            // first lanes, the window's own system)
            float q = 0.f;
            {
                float r1[kF4Seg];
#pragma unroll
                for (int e = 0; e < kF4Seg; ++e) r1[e] = dpp<kWaveShr1>(0.f, rc[e]);
                const float r2a = dpp<kWaveShr1>(0.f, r1[2]);
                const float r2b = dpp<kWaveShr1>(0.f, r1[3]);
                (void)pivot_step<float>(r2a, q);
                (void)pivot_step<float>(r2b, q);
#pragma unroll
                for (int e = 0; e < kF4Seg; ++e) (void)pivot_step<float>(r1[e], q);
            }
            float Ge[kF4Seg], qe[kF4Seg], Qe[kF4Seg];
            float fG, fQ, H, Ev;
            {
                float Gv = 0.f, Qv = 1.f, h = 0.f, ee = 0.f;
#pragma unroll
                for (int e = 0; e < kF4Seg; ++e) {
                    const float m = pivot_step<float>(rc[e], q);
                    const float Pq = Qv;
                    Gv = fma_rn(m, rho[e], q * Gv);
                    Qv = q * Qv;
                    h = fma_rn(Pq, Gv, h);
                    ee = fma_rn(Pq, Qv, ee);
                    Ge[e] = Gv;
                    qe[e] = q;
                    Qe[e] = Qv;
                }
                fG = Gv; fQ = Qv; H = h; Ev = ee;
            }
            float a = fG, b = fQ;
            fu_scan_fwd(a, b);
            const float gin = dpp<kWaveShr1>(0.f, a);
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
            if (lane >= kFuKx / kF4Seg && lane < nl - kFuKx / kF4Seg) {
                // indexed in float4 units, so that each lane's four values are one 16-byte
                // LDS write (contiguous across the wavefront, free of bank conflicts)
                const int o4 = wrap(sb + kFrXr * xw + it) * (kFrS / 4) + (lane - kFuKx / kF4Seg);
                reinterpret_cast<float4*>(sh.w)[o4] = make_float4(wout[0], wout[1], wout[2], wout[3]);
                reinterpret_cast<float4*>(sh.r)[o4] = make_float4(rc[0], rc[1], rc[2], rc[3]);
                reinterpret_cast<float4*>(sh.u)[o4] = make_float4(uc[0], uc[1], uc[2], uc[3]);
            }
        }
    };

    // ---- y-role constants: column c0 + t of the strip (t < wt)
    const bool ycol = t < wt && c0 + t < nx;
    const int lim = (int)(npts * 4);
    const rsrc_t rup = buf(static_cast<const float*>(A.up), lim);
    float gcar = 0.f, qcar = 0.f;                           // forward carries of the column
    float pu[kFrB];                                          // u^{n-1} of the next band's output rows
    // the update operands and results of output row o of band b (row xb - 8 + o):
    // the column's byte offset in a VGPR (out of range for threads past the strip)
    // and the row's in the scalar offset; rows outside the band's output rows are
    // loaded clamped into the grid (unused) and not stored (a uniform test)
    const int vcol = ycol ? (c0 + t) * 4 : kFuOOB;
    const int rowb = nx * 4;
    auto out_row = [&](int b, int o) {
        const int j = xr_lo + kFrB * b - kFuKy + o;
        return j >= max(r0, xr_lo + kFrB * b - kFuKy) && j < min(r1, xr_lo + kFrB * b + 2 * kFuKy);
    };
    auto srow = [&](int b, int o) {
        const int j = xr_lo + kFrB * b - kFuKy + o;
        return (j < 0 ? 0 : j >= ny ? ny - 1 : j) * rowb;
    };
    // a band whose 24 output rows all lie inside the segment (most of them) takes a
    // path with no per-row bound tests or clamps; both paths issue the same loads
    auto band_full = [&](int b) {
        const int j0 = xr_lo + kFrB * b - kFuKy;
        return j0 >= r0 && j0 + kFrB <= r1;
    };
    auto load_upd = [&](int b) {
        if (band_full(b)) {
            const int so0 = (xr_lo + kFrB * b - kFuKy) * rowb;
#pragma unroll
            for (int o = 0; o < kFrB; ++o)
                pu[o] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rup, vcol, so0 + o * rowb, kFuNT));
        } else {
#pragma unroll
            for (int o = 0; o < kFrB; ++o)
                pu[o] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rup, vcol, srow(b, o), kFuNT));
        }
    };
    // band b: its u^{n-1} (requested one pass earlier) is taken first, and band
    // b+1's is requested at once, so that it has a whole pass to arrive;
    // then the forward elimination over the band's rows (g and the pivots replace
    // w and r in the ring), and the back substitution with the update
    auto y_band = [&](int b, int s0) {
        const int xb = xr_lo + kFrB * b;
        float base[kFrB];                                    // -u^{n-1} of the output rows
#pragma unroll
        for (int o = 0; o < kFrB; ++o) base[o] = -pu[o];
        load_upd(b + 1);                                     // past the last band: out of range
        // ring slot s (< 2 kFrR) of this column; threads past the strip read a valid
        // column and write nothing, so every thread issues the same memory operations
        const int ty = t < wt ? t : wt - 1;
        auto at = [&](int s) { return (s >= kFrR ? s - kFrR : s) * kFrS + ty; };
        constexpr int kG = 8;                                // rows per group of LDS reads
#pragma unroll
        for (int c = 0; c < kFrB / kG; ++c) {
            float rr[kG], ww[kG];
#pragma unroll
            for (int e = 0; e < kG; ++e) {
                rr[e] = sh.r[at(s0 + kG * c + e)];
                ww[e] = sh.w[at(s0 + kG * c + e)];
            }
#pragma unroll
            for (int e = 0; e < kG; ++e) {
                const float m = pivot_step<float>(rr[e], qcar);
                gcar = fma_rn(m, ww[e], qcar * gcar);
                if (t < wt) {
                    sh.w[at(s0 + kG * c + e)] = gcar;
                    sh.r[at(s0 + kG * c + e)] = qcar;
                }
            }
        }
        // back substitution from the band's last row, up through the look-ahead rows
        // of the band before (rows xb - 8 .. xb - 1; band 0 has none: zeros, and its
        // rows there are above the strip, so nothing is stored for them)
        const int sl = wrap(s0 + kFrR - kFuKy);                // the slot of row xb - 8
        const int so0 = (xb - kFuKy) * rowb;
        auto back = [&](auto full_c) {
            constexpr bool kFull = decltype(full_c)::value;
            float d = 0.f;
#pragma unroll
            for (int c = 0; c < (kFrB + kFuKy) / kG; ++c) {
                // group c covers rows xb + 16 - 8c .. xb + 23 - 8c (c = 3: the look-ahead rows)
                const bool prev = c == kFrB / kG;
                const int sg = prev ? sl : s0 + kFrB - kG * (c + 1);
                float gg[kG], qq[kG], uu[kG];
#pragma unroll
                for (int e = 0; e < kG; ++e) {
                    gg[e] = sh.w[at(sg + e)];
                    qq[e] = sh.r[at(sg + e)];
                    uu[e] = sh.u[at(sg + e)];
                    if (prev && b == 0) { gg[e] = 0.f; qq[e] = 0.f; }
                }
                const int o0 = kFrB - kG * c;                       // output index of the group's first row
#pragma unroll
                for (int e = kG - 1; e >= 0; --e) {
                    d = fma_rn(qq[e], d, gg[e]);
                    const int o = o0 + e;                           // rows xb - 8 + o
                    if (o < kFrB && (kFull || out_row(b, o))) {
                        const float v = fma_rn(2.f, uu[e], base[o]) + d;
                        const int so = kFull ? so0 + o * rowb : srow(b, o);
                        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), rup, vcol, so, kFuNT);
                    }
                }
            }
        };
        if (band_full(b)) back(std::true_type{});
        else back(std::false_type{});
    };

    // pass k: the x-role solves band k, the y-role band k - 1.  The two roles run
    // separate loops over the same passes (the x-role two passes per iteration, the
    // y-role one), each meeting one barrier per pass: nb + 2 barriers for even nb,
    // nb + 1 for odd, after the one above.  Every wavefront thus meets the same
    // barriers, and each role has its own registers.
    if (wv < kFrY) {
        // one barrier per pass: pass 0 (band 0 being solved), then band b in pass
        // b + 1, and a last barrier when the x-role's loop makes an odd count
        load_upd(0);
        __syncthreads();
        int sb = 0;
        for (int b = 0; b < nb; ++b) {
            y_band(b, sb);
            sb = next_base(sb);
            __syncthreads();
        }
        if ((nb & 1) == 0) __syncthreads();
    } else {
        // the loads are issued on every path (rows past the strip's last band read
        // as zero or are never used), so the outstanding-load count is the same at
        // every point of the loop and each wait covers only the band it needs
        FRIn PA, PB;
        load_band(0, PA);
        load_band(1, PB);
        int sb = 0;
        for (int k = 0; k <= nb; k += 2) {
            if (k < nb) x_band(k, sb, PA);
            sb = next_base(sb);
            load_band(k + 2, PA);
            __syncthreads();
            if (k + 1 < nb) x_band(k + 1, sb, PB);
            sb = next_base(sb);
            load_band(k + 3, PB);
            __syncthreads();
        }
    }
}

}  // namespace adw
