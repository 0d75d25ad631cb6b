// fusedr.hpp -- the one-pass step on column strips with the work split by role,
// so that the y-lines run while the next x-rows are solved and loaded; FP32 and
// FP64 (the constants of each are in FrCfg).  Included by adiwave.hip after
// fused4.hpp, whose x-row scheme it uses.
//
// A workgroup owns a strip of Wt output columns (a multiple of 8, at most S; the
// plan mixes two widths 8 apart so that the strips cover the grid evenly) and hs
// output rows, and walks down it in bands of B x-rows; band k holds the x-rows
// [r0 - KY + Bk, r0 - KY + B + Bk).  (FP32: B = 24, NPL = 4 nodes per lane,
// KX = KY = 8 halo columns and rows, S = 240; FP64: B = 24, NPL = 2, KX = KY = 16,
// S = 64.)
//   x-role (XW = 12 wavefronts): XR = B / XW = 2 x-rows each per band, NPL nodes
//     per lane, on the window [c0 - KX, c0 + Wt + KX) as fused4.hpp, except for the
//     entry pivots (below); w, r and u^n of the central columns go to rings in LDS.
//     The inputs of band k + 1 are in registers, and those of band k + 2 are
//     requested as soon as band k is solved.
//   Entry pivots (FP32): each lane rebuilds the elimination pivot entering its
//     nodes by running the pivot map q -> r / (1 + r (2 - q)) from q = 0 over the
//     PB = 6 nodes before them, instead of reading the full-line value.  The map
//     contracts by its derivative q^2 <= qs^2, so the start value is forgotten to
//     qs^(2 PB + 1), below 1e-11 (qs < 0.14, r <= 0.18): the pivot is the full-line
//     one up to rounding.  The window's first lanes have fewer nodes before them
//     inside the window and start from zero at its edge: that is the window's own
//     system, the same truncation as the y-lines', covered by the bound of fused.hpp
//     (the cut is KX + 1 columns from the first output column).  FP64 would need
//     about nine nodes, four 2-node lanes back, to forget the start to its rounding:
//     its lanes read their full-line entry pivots from a plane of one value per
//     2-node lane (the full-line elimination with the carry entering the window set
//     to zero, the tiles' truncation, under the same bound).
//   y-role (one thread per column): in the same pass, band k - 1.
//     The forward elimination of each y-line continues down the strip from row
//     r0 - KY (zero carries: the upper cut, KY + 1 rows above the first output row),
//     over the band's B rows (g and the pivots replace w and r in the ring).  The
//     back substitution starts at the band's last row with a zero value (the lower
//     cut, KY + 1 rows below the band's last output row), runs up through the band
//     and through the KY look-ahead rows kept in the ring by the band before, and
//     updates the output rows [r0 - 2 KY + Bk, r0 - 2 KY + B + Bk) (band 0:
//     [r0, r0 + B - KY)) as it goes: u^{n+1} = 2 u^n - u^{n-1} + d, with u^n from
//     its ring (the x-role had it in registers) and u^{n-1} requested a pass ahead.
//     The band's last KY rows (g, pivots and u^n) stay in the rings.
//     FP32: YW = 4 wavefronts side by side, each stage in turn.  FP64 (YSPLIT): a
//     64-column strip and one wavefront per stage, so that the two dependency
//     chains of a column (the pivot recurrence with its reciprocal, and the back
//     substitution) run at once: in pass k the elimination wavefront takes band
//     k - 1 and the back-substitution wavefront band k - 2.
// Each output row is the solution of a y-window whose cuts are at least KY + 1 rows
// away, and each x-row that of an x-window cut KX + 1 columns away, so one step
// differs from the exact two-pass step by at most 4 qs^(K+1) max|w| (the bound of
// fused.hpp with K = KX = KY), which the host keeps below half an ulp of the
// arithmetic (2^-24 for FP32 with K = 8, 2^-53 for FP64 with K = 16).  A barrier
// separates the passes: the ring's 2B + KY rows hold the band being solved (B),
// the band being eliminated (B) and the look-ahead rows before it (KY), and these
// never overlap; with the y-role split by stage it has 3B + KY rows, one more band
// for the back substitution.

namespace adw {

template <typename T> struct FrCfg;
template <> struct FrCfg<float> {
    static constexpr int B = 24;           // x-rows per band
    static constexpr int NPL = kF4Seg;     // nodes per lane (one 16-byte vector)
    static constexpr int KX = kFuKx;       // x-halo columns on each side
    static constexpr int KY = kFuKy;       // y-halo rows (look-ahead rows of a band)
    static constexpr int YW = 4;           // y-role wavefronts (one thread per column)
    static constexpr int XW = 12;          // x-role wavefronts (8 with three x-rows each measured slower)
    static constexpr int PB = 6;           // nodes a lane rebuilds its entry pivot over
    static constexpr int KG = 8;           // y-role rows per group of LDS reads
    static constexpr bool YSPLIT = false;  // the y-role's wavefronts share the strip's columns
};
template <> struct FrCfg<double> {
    static constexpr int B = 24;           // 12 x-role wavefronts of two x-rows
    static constexpr int NPL = 2;
    static constexpr int KX = 16;
    static constexpr int KY = 16;
    static constexpr int YW = 2;           // one elimination and one back-substitution wavefront
    static constexpr int XW = 12;          // 896 threads: up to 128 registers a thread
    static constexpr int PB = 8;           // not used: the lanes read their entry pivots
    static constexpr int KG = 8;
    static constexpr bool YSPLIT = true;   // the y-role split by stage, strips of at most 64 columns
};

constexpr int kFrHmin = 256;               // shortest strip segment the plan picks by itself

template <typename T>
struct Fr {
    using C = FrCfg<T>;
    static constexpr int XR = C::B / C::XW;                    // x-rows per x-role wavefront per band (2)
    static_assert(C::B % C::XW == 0, "every x-role wavefront takes the same number of x-rows");
    // ring rows: the band being solved, the band being eliminated and the look-ahead
    // rows before it; with the y-role split by stage also the band being substituted
    // back (56 / 88)
    static constexpr int R = (C::YSPLIT ? 3 : 2) * C::B + C::KY;
    static constexpr int YC = C::YSPLIT ? 1 : C::YW;           // y-role wavefronts across the strip
    static_assert(!C::YSPLIT || C::YW == 2, "a split y-role has one wavefront per stage");
    // ring row stride, widest strip: the x-window's central columns, at most one per
    // y-role thread (240 / 64)
    static constexpr int S = 64 * C::NPL - 2 * C::KX < 64 * YC ? 64 * C::NPL - 2 * C::KX : 64 * YC;
    static constexpr int THREADS = 64 * (C::YW + C::XW);       // workgroup size (1024 / 896)
    static constexpr int LB = (C::PB + C::NPL - 1) / C::NPL;   // lanes the pivot rebuild reaches back
    static constexpr int FIRST = LB * C::NPL - C::PB;          // nodes of the furthest of them skipped
    static_assert(C::B % C::KG == 0 && C::KY % C::KG == 0, "the y-role reads whole groups of rows");
    static_assert(C::KX % C::NPL == 0, "the x-halo is whole lanes");
};
constexpr int kFrThreads = Fr<float>::THREADS;
constexpr int kFrS = Fr<float>::S;          // widest FP32 strip (240)
constexpr int kFrS64 = Fr<double>::S;       // widest FP64 strip (64)
constexpr int kFrThreads64 = Fr<double>::THREADS;

template <typename T>
struct FRShared {
    alignas(16) T w[Fr<T>::R * Fr<T>::S];   // w of the x-rows, then g once the y-role has eliminated them
    alignas(16) T r[Fr<T>::R * Fr<T>::S];   // r of the x-rows, then the y-lines' pivots
    alignas(16) T u[Fr<T>::R * Fr<T>::S];   // u^n of the x-rows, read again by the update
    T src_add[kFuSrc];
    int src_row[kFuSrc];
    int src_wc[kFuSrc];
    int src_n;              // -1: more than kFuSrc in this strip
};

static_assert(sizeof(FRShared<float>) <= 160 * 1024, "the FP32 strip ring exceeds the LDS of a workgroup");
static_assert(sizeof(FRShared<double>) <= 160 * 1024, "the FP64 strip ring exceeds the LDS of a workgroup");

// x-role inputs of one band: u^n rows j-1 .. j+XR and r rows j .. j+XR-1 of the
// wavefront's x-rows, with the window-edge values
template <typename T>
struct FRIn {
    T u[Fr<T>::XR + 2][FrCfg<T>::NPL];
    T e[Fr<T>::XR + 2];
    T r[Fr<T>::XR][FrCfg<T>::NPL];
    T q[Fr<T>::XR];      // FP64: the lane's full-line entry pivot of each x-row
};

// NPL values of T at byte offset vo + so through a buffer resource (16 bytes)
template <typename T>
__device__ __forceinline__ void fr_load_vec(rsrc_t rs, int vo, int so, T (&v)[FrCfg<T>::NPL])
{
    if constexpr (sizeof(T) == 4) {
        const f32x4 x = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, vo, so, 0));
        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    } else {
        const f64x2 x = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(rs, vo, so, 0));
        v[0] = x.x; v[1] = x.y;
    }
}
// one value (AUX: the buffer cache policy bits)
template <typename T, int AUX>
__device__ __forceinline__ T fr_load1(rsrc_t rs, int vo, int so)
{
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, vo, so, AUX));
    else
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, vo, so, AUX));
}
template <typename T, int AUX>
__device__ __forceinline__ void fr_store1(T v, rsrc_t rs, int vo, int so)
{
    if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), rs, vo, so, AUX);
    } else {
        using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(rs, 0, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), rs, vo, so, AUX);
    }
}
// one lane's NPL values of a ring row as one 16-byte LDS write (v4 indexes 16-byte units)
template <typename T>
__device__ __forceinline__ void fr_put_vec(T* ring, int v4, const T (&v)[FrCfg<T>::NPL])
{
    if constexpr (sizeof(T) == 4)
        reinterpret_cast<float4*>(ring)[v4] = make_float4(v[0], v[1], v[2], v[3]);
    else
        reinterpret_cast<double2*>(ring)[v4] = make_double2(v[0], v[1]);
}

// inclusive suffix (lanes l..63) of two-component affine maps over the wavefront
// (FP32: wave_scan_bwd2 of fused.hpp)
template <typename T>
__device__ __forceinline__ void fr_scan_bwd2(T& a, T& b, int lane)
{
    if constexpr (sizeof(T) == 4) {
        wave_scan_bwd2(a, b, lane);
    } else {
        row_scan_bwd(a, b);
        const T a16 = readlane(a, 16), b16 = readlane(b, 16);
        const T a32 = readlane(a, 32), b32 = readlane(b, 32);
        const T a48 = readlane(a, 48), b48 = readlane(b, 48);
        const T a23 = fma_rn(b32, a48, a32), b23 = b32 * b48;
        const T a13 = fma_rn(b16, a23, a16), b13 = b16 * b23;
        T ca = T(0), cb = T(1);
        if (lane < 16) { ca = a13; cb = b13; }
        else if (lane < 32) { ca = a23; cb = b23; }
        else if (lane < 48) { ca = a48; cb = b48; }
        a = fma_rn(b, ca, a);
        b = b * cb;
    }
}

// One strip segment (blk = segment row * tiles_x + strip) of the grid A
// describes, by the whole workgroup.
template <typename T>
__device__ __forceinline__ void fusedr_strip(const FArgsT<T>& A, int blk, FRShared<T>& sh)
{
    using C = FrCfg<T>;
    constexpr int NPL = C::NPL, KX = C::KX, KY = C::KY, KG = C::KG, kFrB = C::B;
    constexpr int R = Fr<T>::R, S = Fr<T>::S, XR = Fr<T>::XR;
    constexpr int ES = (int)sizeof(T);
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int nx = A.nx, ny = A.ny;
    const int sx = blk % A.tiles_x;                       // strip index: the first A.wide are
    const int wt = sx < A.wide ? A.wt : A.wt - 8;         // A.wt wide, the others 8 narrower
    const int c0 = sx * A.wt - (sx > A.wide ? (sx - A.wide) * 8 : 0);
    const int r0 = (blk / A.tiles_x) * A.hs;
    const int r1 = min(r0 + A.hs, ny);
    // bands: band b outputs rows [r0 - 2 KY + B b, r0 - 2 KY + B + B b), so
    // B nb >= hs + 2 KY
    const int nb = (r1 - r0 + 2 * KY + kFrB - 1) / kFrB;
    const int nl = (wt + 2 * KX) / NPL;                   // lanes of the x-window
    const long long npts = (long long)nx * ny;
    const int xr_lo = r0 - KY, xr_hi = xr_lo + kFrB * nb;   // x-rows of the strip
    // ring slot of x-row xr_lo + B k + i (0 <= i < R): the band's first slot
    // (B k mod R) is carried from band to band, so no division is needed
    auto wrap = [](int s) { return s >= R ? s - R : s; };
    auto next_base = [&](int sb) { return wrap(sb + kFrB); };

    // ---- point sources of the strip's x-rows and x-window, in source order
    if (t < 64) {
        int n = 0;
        for (int base = 0; base < A.nsrc; base += 64) {
            const int qq = base + t;
            int id = -1;
            T amp = T(0);
            if (qq < A.nsrc) { id = A.src_idx[qq]; amp = A.src_amp[qq]; }
            const int row = (id >= 0 && id < npts) ? id / nx : -1;
            const int col = row >= 0 ? id - row * nx : 0;
            const int wc = col - (c0 - KX);
            const bool hit = row >= 0 && row >= xr_lo && row < xr_hi && wc >= 0 && wc < nl * NPL;
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
    const int row_bytes = nx * ES;
    auto row_ok = [&](int j) { return j >= 0 && j < ny; };

    // ---- x-role constants
    const int xw = wv - C::YW;                              // x-role wavefront index
    const bool inwin = lane < nl;
    const int col0 = c0 - KX + lane * NPL;                  // first column of the lane
    // One buffer resource per plane: a row is reached through the scalar offset, and
    // whatever lies outside the grid (the lanes or edge values past a wall, whole rows
    // above or below it, the bands past the strip's last) through a vector offset past
    // every range, which the range check turns into zeros without a memory access.
    const int ecol = (lane == 0) ? c0 - KX - 1 : (lane == nl - 1) ? c0 + wt + KX : -1;
    const int voff = (inwin && col0 >= 0 && col0 < nx) ? col0 * ES : kFuOOB;
    const int eoff = (ecol >= 0 && ecol < nx) ? ecol * ES : kFuOOB;
    const int plane = (int)(npts * ES);
    const rsrc_t ru_all = buf(A.uc, plane);
    const rsrc_t rr_all = buf(A.r, plane);
    // FP64: A.qin holds the entry pivot of every 2-node lane, ceil(nx / 2) a row (nx is even)
    const rsrc_t rq_all = buf(A.qin, sizeof(T) == 8 ? (int)(npts / 2 * ES) : 0);
    const int qoff = voff == kFuOOB ? kFuOOB : voff / 2;
    // pieces of band k's inputs: u^n row j-1+i (with its window-edge values), and
    // r row j+i, j = the wavefront's first x-row of band k
    auto load_u = [&](int k, int i, FRIn<T>& P) {
        const int jj = xr_lo + kFrB * k + XR * xw - 1 + i;
        const bool ok = row_ok(jj) && k < nb;
        const int so = ok ? jj * row_bytes : 0;
        fr_load_vec<T>(ru_all, ok ? voff : kFuOOB, so, P.u[i]);
        P.e[i] = fr_load1<T, 0>(ru_all, ok ? eoff : kFuOOB, so);
    };
    auto load_r = [&](int k, int i, FRIn<T>& P) {
        const int jj = xr_lo + kFrB * k + XR * xw + i;
        const bool ok = row_ok(jj) && k < nb;
        fr_load_vec<T>(rr_all, ok ? voff : kFuOOB, ok ? jj * row_bytes : 0, P.r[i]);
        if constexpr (sizeof(T) == 8) P.q[i] = fr_load1<T, 0>(rq_all, ok ? qoff : kFuOOB, ok ? jj * (row_bytes / 2) : 0);
    };
    auto load_band = [&](int k, FRIn<T>& P) {
#pragma unroll
        for (int i = 0; i < XR + 2; ++i) load_u(k, i, P);
#pragma unroll
        for (int i = 0; i < XR; ++i) load_r(k, i, P);
    };
    // the x-rows of band k from P (sb: the band's first ring slot); w and r of the
    // central columns to the ring.  The wavefront's XR rows are independent: each
    // stage below runs for all of them before the next, so that their dependency
    // chains (the pivot recurrences, the scans) interleave.
    auto x_band = [&](int k, int sb, const FRIn<T>& P) {
        T rho[XR][NPL];
#pragma unroll
        for (int it = 0; it < XR; ++it) {
            const int j = xr_lo + kFrB * k + XR * xw + it;
            const T(&um)[NPL] = P.u[it];
            const T(&uc)[NPL] = P.u[it + 1];
            const T(&u1)[NPL] = P.u[it + 2];
            const T(&rc)[NPL] = P.r[it];
            const T eC = P.e[it + 1];
            {
                const T west = dpp<kWaveShr1>(T(0), uc[NPL - 1]);
                const T east = dpp<kWaveShl1>(T(0), uc[0]);
                const T w0 = lane == 0 ? eC : west;
                const T eL = lane == nl - 1 ? eC : east;
#pragma unroll
                for (int e = 0; e < NPL; ++e) {
                    const T uw = e == 0 ? w0 : uc[e - 1];
                    const T ue = e == NPL - 1 ? eL : uc[e + 1];
                    rho[it][e] = T(2) * (rc[e] * (((uw + ue) + (um[e] + u1[e])) - T(4) * uc[e]));
                }
            }
            if (ns > 0) {
                for (int s = 0; s < ns; ++s) {
                    if (sh.src_row[s] == j) {
                        const int i = sh.src_wc[s] - lane * NPL;
                        const T add = sh.src_add[s];
#pragma unroll
                        for (int e = 0; e < NPL; ++e)
                            if (e == i) rho[it][e] += add;
                    }
                }
            } else if (ns < 0 && row_ok(j)) {
                for (int s = 0; s < A.nsrc; ++s) {
                    const int id = A.src_idx[s];
                    if (id >= 0 && id < npts && id / nx == j) {
                        const int i = id - j * nx - col0;
                        const T add = A.tau2 * A.src_amp[s];
#pragma unroll
                        for (int e = 0; e < NPL; ++e)
                            if (e == i && inwin) rho[it][e] += add;
                    }
                }
            }
        }
        // entry pivot of each lane: FP64 reads the full-line pivot; FP32 rebuilds it
        // from zero over the PB nodes before the lane (see the header: within rounding
        // of the full-line pivot; at the window's first lanes, the window's own
        // system): rb[b] holds r of the lane b + 1 places to the left; the furthest
        // lane's first FIRST nodes are not used
        T q[XR];
        if constexpr (sizeof(T) == 8) {
#pragma unroll
            for (int it = 0; it < XR; ++it) q[it] = P.q[it];
        } else {
            constexpr int LB = Fr<T>::LB, FIRST = Fr<T>::FIRST;
            T rb[XR][LB][NPL];
#pragma unroll
            for (int it = 0; it < XR; ++it) {
                q[it] = T(0);
#pragma unroll
                for (int e = 0; e < NPL; ++e) rb[it][0][e] = dpp<kWaveShr1>(T(0), P.r[it][e]);
#pragma unroll
                for (int b = 1; b < LB; ++b)
#pragma unroll
                    for (int e = 0; e < NPL; ++e)
                        rb[it][b][e] = (b == LB - 1 && e < FIRST) ? T(0) : dpp<kWaveShr1>(T(0), rb[it][b - 1][e]);
            }
#pragma unroll
            for (int b = LB - 1; b >= 0; --b)
#pragma unroll
                for (int e = (b == LB - 1 ? FIRST : 0); e < NPL; ++e)
#pragma unroll
                    for (int it = 0; it < XR; ++it) (void)pivot_step<T>(rb[it][b][e], q[it]);
        }
        // local elimination of each lane's nodes, then the scans across the line
        T Ge[XR][NPL], qe[XR][NPL], Qe[XR][NPL], fG[XR], fQ[XR], H[XR], Ev[XR];
        {
            T Gv[XR], Qv[XR], hh[XR], ee[XR];
#pragma unroll
            for (int it = 0; it < XR; ++it) { Gv[it] = T(0); Qv[it] = T(1); hh[it] = T(0); ee[it] = T(0); }
#pragma unroll
            for (int e = 0; e < NPL; ++e) {
#pragma unroll
                for (int it = 0; it < XR; ++it) {
                    const T m = pivot_step<T>(P.r[it][e], q[it]);
                    const T Pq = Qv[it];
                    Gv[it] = fma_rn(m, rho[it][e], q[it] * Gv[it]);
                    Qv[it] = q[it] * Qv[it];
                    hh[it] = fma_rn(Pq, Gv[it], hh[it]);
                    ee[it] = fma_rn(Pq, Qv[it], ee[it]);
                    Ge[it][e] = Gv[it];
                    qe[it][e] = q[it];
                    Qe[it][e] = Qv[it];
                }
            }
#pragma unroll
            for (int it = 0; it < XR; ++it) { fG[it] = Gv[it]; fQ[it] = Qv[it]; H[it] = hh[it]; Ev[it] = ee[it]; }
        }
        T gin[XR], ba[XR], bb[XR];
#pragma unroll
        for (int it = 0; it < XR; ++it) {
            T a = fG[it], b = fQ[it];
            wave_scan_fwd(a, b);
            gin[it] = dpp<kWaveShr1>(T(0), a);
            ba[it] = inwin ? fma_rn(Ev[it], gin[it], H[it]) : T(0);
            bb[it] = inwin ? fQ[it] : T(1);
        }
#pragma unroll
        for (int it = 0; it < XR; ++it) fr_scan_bwd2<T>(ba[it], bb[it], lane);
#pragma unroll
        for (int it = 0; it < XR; ++it) {
            const T dbelow = dpp<kWaveShl1>(T(0), ba[it]);
            T wout[NPL];
            {
                T x = dbelow;
#pragma unroll
                for (int e = NPL - 1; e >= 0; --e) {
                    x = fma_rn(qe[it][e], x, fma_rn(Qe[it][e], gin[it], Ge[it][e]));
                    wout[e] = x;
                }
            }
            if (lane >= KX / NPL && lane < nl - KX / NPL) {
                // indexed in 16-byte units, so that each lane's values are one 16-byte
                // LDS write (contiguous across the wavefront, free of bank conflicts)
                const int o4 = wrap(sb + XR * xw + it) * (S / NPL) + (lane - KX / NPL);
                fr_put_vec<T>(sh.w, o4, wout);
                fr_put_vec<T>(sh.r, o4, P.r[it]);
                fr_put_vec<T>(sh.u, o4, P.u[it + 1]);
            }
        }
    };

    // ---- y-role constants: column c0 + yt of the strip (yt < wt); yt is the thread
    // within the y-role, or within its stage's wavefront when the y-role is split
    const int yt = C::YSPLIT ? lane : t;
    const bool ycol = yt < wt && c0 + yt < nx;
    const int lim = (int)(npts * ES);
    const rsrc_t rup = buf(static_cast<const T*>(A.up), lim);
    T gcar = T(0), qcar = T(0);                              // forward carries of the column
    T pu[kFrB];                                              // u^{n-1} of the next band's output rows
    // the update operands and results of output row o of band b (row xb - KY + o):
    // the column's byte offset in a VGPR (out of range for threads past the strip)
    // and the row's in the scalar offset; rows outside the band's output rows are
    // loaded clamped into the grid (unused) and not stored (a uniform test)
    const int vcol = ycol ? (c0 + yt) * ES : kFuOOB;
    const int rowb = nx * ES;
    auto out_row = [&](int b, int o) {
        const int j = xr_lo + kFrB * b - KY + o;
        return j >= max(r0, xr_lo + kFrB * b - KY) && j < min(r1, xr_lo + kFrB * b - KY + kFrB);
    };
    auto srow = [&](int b, int o) {
        const int j = xr_lo + kFrB * b - KY + o;
        return (j < 0 ? 0 : j >= ny ? ny - 1 : j) * rowb;
    };
    // a band whose B output rows all lie inside the segment (most of them) takes a
    // path with no per-row bound tests or clamps; both paths issue the same loads
    auto band_full = [&](int b) {
        const int j0 = xr_lo + kFrB * b - KY;
        return j0 >= r0 && j0 + kFrB <= r1;
    };
    auto load_upd = [&](int b) {
        if (band_full(b)) {
            const int so0 = (xr_lo + kFrB * b - KY) * rowb;
#pragma unroll
            for (int o = 0; o < kFrB; ++o) pu[o] = fr_load1<T, kFuNT>(rup, vcol, so0 + o * rowb);
        } else {
#pragma unroll
            for (int o = 0; o < kFrB; ++o) pu[o] = fr_load1<T, kFuNT>(rup, vcol, srow(b, o));
        }
    };
    // band b from ring slot s0, in two stages: the forward elimination over the
    // band's rows (g and the pivots replace w and r in the ring), then the back
    // substitution from the band's last row, up through the look-ahead rows of the
    // band before, with the update.  Its u^{n-1} (requested one pass earlier) is
    // taken first, and band b+1's is requested at once, so that it has a whole pass
    // to arrive.  kElim / kBack select the stages (both, or one of them for a
    // y-role split by stage; there the back substitution's wavefront reads u^{n-1}
    // in place and requests band b+1's when it is done, since it finishes its
    // passes early and waits at the barrier).
    auto y_band = [&](int b, int s0, auto elim_c, auto back_c) {
        constexpr bool kElim = decltype(elim_c)::value, kBack = decltype(back_c)::value;
        const int xb = xr_lo + kFrB * b;
        T base[kFrB];                                        // -u^{n-1} of the output rows
        if constexpr (kBack && !C::YSPLIT) {
#pragma unroll
            for (int o = 0; o < kFrB; ++o) base[o] = -pu[o];
            load_upd(b + 1);                                 // past the last band: clamped rows, unused
        }
        // ring slot s (< 2 R) of this column; threads past the strip read a valid
        // column and write nothing, so every thread issues the same memory operations
        const int ty = yt < wt ? yt : wt - 1;
        auto at = [&](int s) { return (s >= R ? s - R : s) * S + ty; };
        if constexpr (kElim && C::YSPLIT) {
            // the band's reads all first, so that the pivot recurrence then runs
            // without waiting on LDS; a thread past the strip repeats the values of
            // column wt - 1 (the same reads from zero carries), so its writes are
            // duplicates and need no test
            T rr[kFrB], ww[kFrB];
#pragma unroll
            for (int e = 0; e < kFrB; ++e) {
                rr[e] = sh.r[at(s0 + e)];
                ww[e] = sh.w[at(s0 + e)];
            }
#pragma unroll
            for (int e = 0; e < kFrB; ++e) {
                const T m = pivot_step<T>(rr[e], qcar);
                gcar = fma_rn(m, ww[e], qcar * gcar);
                sh.w[at(s0 + e)] = gcar;
                sh.r[at(s0 + e)] = qcar;
            }
        } else if constexpr (kElim) {
#pragma unroll
            for (int c = 0; c < kFrB / KG; ++c) {
                T rr[KG], ww[KG];
#pragma unroll
                for (int e = 0; e < KG; ++e) {
                    rr[e] = sh.r[at(s0 + KG * c + e)];
                    ww[e] = sh.w[at(s0 + KG * c + e)];
                }
#pragma unroll
                for (int e = 0; e < KG; ++e) {
                    const T m = pivot_step<T>(rr[e], qcar);
                    gcar = fma_rn(m, ww[e], qcar * gcar);
                    if (yt < wt) {
                        sh.w[at(s0 + KG * c + e)] = gcar;
                        sh.r[at(s0 + KG * c + e)] = qcar;
                    }
                }
            }
        }
        if constexpr (!kBack) return;
        // back substitution from the band's last row, up through the look-ahead rows
        // of the band before (rows xb - KY .. xb - 1; band 0 has none: zeros, and its
        // rows there are above the strip, so nothing is stored for them)
        const int sl = wrap(s0 + R - KY);                    // the slot of row xb - KY
        const int so0 = (xb - KY) * rowb;
        auto back = [&](auto full_c) {
            constexpr bool kFull = decltype(full_c)::value;
            T d = T(0);
#pragma unroll
            for (int c = 0; c < (kFrB + KY) / KG; ++c) {
                // group c covers rows xb + B - KG (c + 1) .. xb + B - 1 - KG c; the
                // groups from c = B / KG on are the look-ahead rows
                const bool prev = c >= kFrB / KG;
                const int sg = prev ? sl + KY - KG * (c - kFrB / KG + 1) : s0 + kFrB - KG * (c + 1);
                T gg[KG], qq[KG], uu[KG];
#pragma unroll
                for (int e = 0; e < KG; ++e) {
                    gg[e] = sh.w[at(sg + e)];
                    qq[e] = sh.r[at(sg + e)];
                    uu[e] = sh.u[at(sg + e)];
                    if (prev && b == 0) { gg[e] = T(0); qq[e] = T(0); }
                }
                const int o0 = kFrB + KY - KG * (c + 1);            // output index of the group's first row
#pragma unroll
                for (int e = KG - 1; e >= 0; --e) {
                    d = fma_rn(qq[e], d, gg[e]);
                    const int o = o0 + e;                           // rows xb - KY + o
                    if (o < kFrB && (kFull || out_row(b, o))) {
                        const T v = fma_rn(T(2), uu[e], C::YSPLIT ? -pu[o] : base[o]) + d;
                        const int so = kFull ? so0 + o * rowb : srow(b, o);
                        fr_store1<T, kFuNT>(v, rup, vcol, so);
                    }
                }
            }
        };
        if (band_full(b)) back(std::true_type{});
        else back(std::false_type{});
        if constexpr (C::YSPLIT) load_upd(b + 1);        // past the last band: clamped rows, unused
    };

    // pass k: the x-role solves band k and the y-role band k - 1 (split by stage:
    // the elimination of band k - 1 and the back substitution of band k - 2).  The
    // roles run separate loops over the same passes (the x-role two passes per
    // iteration, the y-role one), each meeting one barrier per pass, and one more
    // when the x-role's loop makes an odd count, after the one above.  Every
    // wavefront thus meets the same barriers, and each role has its own registers.
    const int npass = nb + (C::YSPLIT ? 2 : 1);
    if (wv < C::YW) {
        int sb = 0;
        if constexpr (C::YSPLIT) {
            if (wv == 0) {
                // elimination of band b in pass b + 1
                __syncthreads();
                for (int b = 0; b < nb; ++b) {
                    y_band(b, sb, std::true_type{}, std::false_type{});
                    sb = next_base(sb);
                    __syncthreads();
                }
            } else {
                // back substitution of band b in pass b + 2, with its u^{n-1}
                // requested a pass ahead
                load_upd(0);
                __syncthreads();
                __syncthreads();
                for (int b = 0; b < nb; ++b) {
                    y_band(b, sb, std::false_type{}, std::true_type{});
                    sb = next_base(sb);
                    __syncthreads();
                }
            }
            if (wv == 0) __syncthreads();                     // pass nb + 1
        } else {
            // pass 0 (band 0 being solved), then band b in pass b + 1
            load_upd(0);
            __syncthreads();
            for (int b = 0; b < nb; ++b) {
                y_band(b, sb, std::true_type{}, std::true_type{});
                sb = next_base(sb);
                __syncthreads();
            }
        }
        if (npass & 1) __syncthreads();
    } else {
        // the loads are issued on every path (rows past the strip's last band read
        // as zero or are never used), so the outstanding-load count is the same at
        // every point of the loop and each wait covers only the band it needs
        FRIn<T> PA, PB;
        load_band(0, PA);
        load_band(1, PB);
        int sb = 0;
        for (int k = 0; k < npass; k += 2) {
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

template <typename T>
__global__ void __launch_bounds__(Fr<T>::THREADS) k_fusedr(FArgsT<T> A)
{
    __shared__ FRShared<T> sh;
    rec_tap<T>(A.uc, A.rec_idx, A.rec_out, A.nrec, (long long)A.nx * A.ny);
    // neighbouring strips of a segment row run on one XCD (their halo columns meet
    // in that XCD's L2): the grid is a multiple of 8 and blocks past the tiles exit
    const int blk = A.xcd_map ? xcd_band(blockIdx.x) : (int)blockIdx.x;
    if (blk >= A.tiles) return;
    fusedr_strip<T>(A, blk, sh);
}

}  // namespace adw
