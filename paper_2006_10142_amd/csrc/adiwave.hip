// adiwave.hip -- C-ABI runtime of the gfx950 ADI wave solver: handles,
// workspace, launch planning, argument validation and error reporting.
// The operations and their layouts are specified in include/adiwave.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "adiwave.h"
#include "kernels.hpp"
#include "fused.hpp"
#include "fused4.hpp"
#include "fusedr.hpp"
#include "cr.hpp"
#include "tridiag_part.hpp"

using namespace adw;

// --------------------------------------------------------------- errors ----
namespace {

thread_local std::string g_err;

adi_status fail(adi_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

#define ADI_HIP(call)                                                                \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess)                                                        \
            return fail(ADI_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define ADI_LAUNCHED(name)                                                           \
    do {                                                                             \
        hipError_t e_ = hipGetLastError();                                           \
        if (e_ != hipSuccess)                                                        \
            return fail(ADI_EHIP, std::string("launch ") + (name) + ": " +           \
                                      hipGetErrorString(e_));                        \
    } while (0)

size_t esize(adi_dtype t) { return t == ADI_F64 ? 8 : 4; }

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// ---------------------------------------------------------- launch plans ----
struct XPlan { int tr, rs, fuse, frs; };   // frs: rows of a fused strip (whole chunks)

// x-sweep: smallest line group whose 8 * tr nodes cover nx
bool choose_x(int nx, adi_dtype, XPlan& p)
{
    static const int cand[] = {64, 128, 256, 1024};
    for (int tr : cand)
        if (8LL * tr >= nx) { p.tr = tr; return true; }
    return false;
}

// the fused y-chunk state (4 values per column) must fit in LDS next to the rest
bool fuse_fits(int tr, adi_dtype dt)
{
    // LDS of one workgroup of the fused x-sweep: G = max(tr, 256) / tr line groups
    auto bytes = [&](auto tag) -> size_t {
        using T = decltype(tag);
        switch (tr) {
        case 64: return 4 * sizeof(XShared<T, 64, true>);
        case 128: return 2 * sizeof(XShared<T, 128, true>);
        case 256: return sizeof(XShared<T, 256, true>);
        case 1024: return sizeof(XShared<T, 1024, true>);
        default: return SIZE_MAX;
        }
    };
    const size_t lds = dt == ADI_F64 ? bytes(double()) : bytes(float());
    return lds <= 150 * 1024;
}

// batched solve: smallest (threads per line, nodes per thread) covering n
struct TPlan { int tr, s; };
bool choose_tri(int n, adi_dtype dt, TPlan& p)
{
    static const int cand[][2] = {{64, 2}, {64, 4}, {64, 8}, {64, 16}, {256, 8},
                                  {256, 16}, {1024, 8}, {1024, 16}};
    for (auto& c : cand) {
        if (dt == ADI_F64 && c[1] > 8) continue;
        if ((long long)c[0] * c[1] >= n) { p.tr = c[0]; p.s = c[1]; return true; }
    }
    return false;
}

int x_groups_per_wg(int tr) { return tr >= 256 ? 1 : 256 / tr; }

// rows per strip: enough workgroups to cover 256 CUs twice, 1..32 rows (the rows
// of a strip are solved one after another, so short strips suit small grids)
int choose_rows(int ny, int tr)
{
    const int g = x_groups_per_wg(tr);
    int rs = ny / (512 * g);
    return std::max(1, std::min(32, rs));
}

struct YScanPlan { int sk, p; };
bool choose_yscan(int K, YScanPlan& q)
{
    static const int cand[][2] = {{16, 2}, {16, 4}, {16, 8}, {64, 4}, {64, 8}};
    for (auto& c : cand)
        if ((long long)c[0] * c[1] >= K) { q.p = c[0]; q.sk = c[1]; return true; }
    return false;
}

// fused strips hold whole y-chunks: 32 rows, or one chunk when chunks are longer
int fused_rows(int M) { return M * std::max(1, 32 / M); }

// ---------------------------------------------------- template dispatch ----
template <typename T, int TR, bool FUSE>
void launch_x1(int grid, const XArgs<T>& a, hipStream_t st)
{
    constexpr int NT = TR >= 256 ? TR : 256;
    hipLaunchKernelGGL((k_xsweep<T, TR, FUSE>), dim3(grid), dim3(NT), 0, st, a);
}

template <typename T, int TR>
bool launch_x_f(bool fuse, int grid, const XArgs<T>& a, hipStream_t st)
{
    if (fuse) {
        if constexpr (sizeof(T) == 8 && TR > 256) return false;
        else { launch_x1<T, TR, true>(grid, a, st); return true; }
    }
    launch_x1<T, TR, false>(grid, a, st);
    return true;
}

template <typename T>
bool launch_x(const XPlan& p, int grid, const XArgs<T>& a, hipStream_t st)
{
    switch (p.tr) {
        case 64: return launch_x_f<T, 64>(p.fuse != 0, grid, a, st);
        case 128: return launch_x_f<T, 128>(p.fuse != 0, grid, a, st);
        case 256: return launch_x_f<T, 256>(p.fuse != 0, grid, a, st);
        case 1024: return launch_x_f<T, 1024>(p.fuse != 0, grid, a, st);
    }
    return false;
}

template <typename T, int P>
bool launch_yscan_sk(int sk, int grid, const YArgs<T>& a, hipStream_t st)
{
    const dim3 blk(kPB * P);
    switch (sk) {
        case 2: hipLaunchKernelGGL((k_yscan<T, 2, P>), dim3(grid), blk, 0, st, a); return true;
        case 4: hipLaunchKernelGGL((k_yscan<T, 4, P>), dim3(grid), blk, 0, st, a); return true;
        case 8: hipLaunchKernelGGL((k_yscan<T, 8, P>), dim3(grid), blk, 0, st, a); return true;
    }
    return false;
}

template <typename T>
bool launch_yscan(const YScanPlan& q, int nx, const YArgs<T>& a, hipStream_t st)
{
    const int grid = (nx + kPB - 1) / kPB;
    switch (q.p) {
        case 16: return launch_yscan_sk<T, 16>(q.sk, grid, a, st);
        case 64: return launch_yscan_sk<T, 64>(q.sk, grid, a, st);
    }
    return false;
}

template <typename T>
bool launch_ysolve(int M, dim3 grid, const YArgs<T>& a, hipStream_t st)
{
    switch (M) {
        case 16: hipLaunchKernelGGL((k_ysolve<T, 16, 16>), grid, dim3(256), 0, st, a); return true;
        case 32: hipLaunchKernelGGL((k_ysolve<T, 32, 8>), grid, dim3(256), 0, st, a); return true;
    }
    return false;
}

template <typename T, int S, int TR>
void launch_tri1(long long batch, const TriArgs<T>& a, hipStream_t st)
{
    constexpr int NT = TR >= 256 ? TR : 256;
    constexpr int G = NT / TR;
    const long long grid = (batch + G - 1) / G;
    hipLaunchKernelGGL((k_tridiag_wg<T, S, TR>), dim3((unsigned)grid), dim3(NT), 0, st, a);
}

template <typename T, int TR>
bool launch_tri_s(int s, long long batch, const TriArgs<T>& a, hipStream_t st)
{
    switch (s) {
        case 2: launch_tri1<T, 2, TR>(batch, a, st); return true;
        case 4: launch_tri1<T, 4, TR>(batch, a, st); return true;
        case 8: launch_tri1<T, 8, TR>(batch, a, st); return true;
        case 16:
            if constexpr (sizeof(T) == 4) { launch_tri1<T, 16, TR>(batch, a, st); return true; }
            return false;
    }
    return false;
}

template <typename T>
bool launch_tri(const TPlan& p, long long batch, const TriArgs<T>& a, hipStream_t st)
{
    switch (p.tr) {
        case 64: return launch_tri_s<T, 64>(p.s, batch, a, st);
        case 256: return launch_tri_s<T, 256>(p.s, batch, a, st);
        case 1024: return launch_tri_s<T, 1024>(p.s, batch, a, st);
    }
    return false;
}

}  // namespace

// --------------------------------------------------------------- handle ----
struct adi_adjoint_s;   // adjoint checkpoint and work storage (adjoint.hpp)

struct adi_wave_s {
    int nx = 0, ny = 0;
    double h = 0, dt = 0;
    adi_dtype dtype = ADI_F32;
    hipStream_t stream = nullptr;
    int device = 0;
    void* r = nullptr;     // nx*ny
    void* w = nullptr;     // nx*ny
    void* sum = nullptr;   // 8 * K * nx
    void* X = nullptr;     // K * nx
    void* qin = nullptr;   // ny * nseg entry pivots of the x-line segments
    void* qin2 = nullptr;  // FP64: ny * ceil(nx / 2) entry pivots of every 2-node lane (one-pass strips)
    int nseg = 0;
    int nxp = 0;           // nx rounded up to the summary-plane column block
    size_t w_cap = 0;      // elements of w (also create-time scratch of 5*K*nx)
    XPlan xp{};
    int M = 32, K = 0;
    YScanPlan yq{};
    size_t bytes = 0;
    adi_adjoint_s* adj = nullptr;   // created by the first adjoint forward run
    // bumped by every coefficient change and every adjoint forward run: the
    // forward run's record id, which a later change invalidates
    unsigned long long gen = 0;
    // one-pass step (FP32): allowed when the truncation bound holds for the
    // largest r; mode 0 = automatic, 1 = on when allowed, 2 = off
    double rmax = 0.0;   // largest r, measured on the device when the coefficient is set
    int fused_ok = 0, fused_mode = 0, fstep = 0;
    int f_wt = 0, f_tx = 0, f_tiles = 0, f_grid = 0;
    int f_wide = 0;      // column strips: the first f_wide are f_wt wide, the others f_wt - 8
    int f_ncu = 0;       // compute units the tiles are balanced over (0: widest tiles)
    int f_wt_user = 0;   // tile width set through adi_wave_set_tuning (0: chosen here)
    int f_lane = 8;      // nodes per lane of the one-pass x-lines (8: fused.hpp, 4: fused4.hpp)
    int f_lane_user = 0; // nodes per lane set through adi_wave_set_tuning (0: chosen here)
    int f_hs = 0;        // output rows per column-strip segment (fusedr.hpp); 0: 64-row tiles
    int f_hs_user = 0;   // set through adi_wave_set_tuning: > 0 strips, -2 tiles, 0 chosen here
    int f4_wt = 0, f4_tx = 0, f4_tiles = 0;   // widest four-node tiles (used by the batched step)
    // cyclic-reduction baseline (line_solver = 2): coefficient arrays a, b, c
    int cr = 0;
    void* cr_abc = nullptr;   // 3 * nx * ny values
    // time-dependent coefficient steps: r at the previous level, right-hand side
    void* r_prev = nullptr;
    void* rho_buf = nullptr;
    // receivers of the previous step, recorded by the next step's first launch
    // (set by do_step around one queued step, empty otherwise)
    int tap_n = 0;
    const int* tap_idx = nullptr;
    void* tap_out = nullptr;
};

namespace {

void adjoint_free(adi_adjoint_s* a);   // adjoint.hpp

void free_ws(adi_wave_s* w)
{
    if (w->r) (void)hipFree(w->r);
    if (w->w) (void)hipFree(w->w);
    if (w->sum) (void)hipFree(w->sum);
    if (w->X) (void)hipFree(w->X);
    if (w->qin) (void)hipFree(w->qin);
    if (w->qin2) (void)hipFree(w->qin2);
    if (w->cr_abc) (void)hipFree(w->cr_abc);
    if (w->r_prev) (void)hipFree(w->r_prev);
    if (w->rho_buf) (void)hipFree(w->rho_buf);
    w->r = w->w = w->sum = w->X = w->qin = w->qin2 = w->cr_abc = w->r_prev = w->rho_buf = nullptr;
}

adi_status alloc_chunks(adi_wave_s* w)
{
    const size_t es = esize(w->dtype);
    if (w->sum) (void)hipFree(w->sum);
    if (w->X) (void)hipFree(w->X);
    w->sum = w->X = nullptr;
    w->K = (w->ny + w->M - 1) / w->M;
    w->nxp = (w->nx + kPB - 1) / kPB * kPB;
    if (!choose_yscan(w->K, w->yq))
        return fail(ADI_EUNSUPPORTED, "too many y-chunks for the interface solver (ny too large)");
    const size_t nsum = (size_t)kSummaryPlanes * w->K * w->nxp;
    const size_t nX = (size_t)w->K * w->nx;
    const size_t wneed = std::max((size_t)w->nx * w->ny, (size_t)5 * w->K * w->nx);
    if (wneed > w->w_cap) {
        if (w->w) (void)hipFree(w->w);
        w->w = nullptr;
        w->w_cap = 0;
        if (hipMalloc(&w->w, wneed * es) != hipSuccess) {
            (void)hipGetLastError();
            w->w = nullptr;
            return fail(ADI_ENOMEM, "hipMalloc of the x-sweep field failed");
        }
        w->w_cap = wneed;
    }
    if (hipMalloc(&w->sum, nsum * es) != hipSuccess || hipMalloc(&w->X, nX * es) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ADI_ENOMEM, "hipMalloc of y-chunk workspace failed");
    }
    w->bytes = ((size_t)w->nx * w->ny + w->w_cap + (size_t)w->ny * w->nseg + nsum + nX +
                (w->qin2 ? (size_t)w->ny * ((w->nx + 1) / 2) : 0)) * es;
    return ADI_OK;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

adi_status check_handle(adi_wave_t w)
{
    if (!w) return fail(ADI_EINVAL, "null handle");
    return ADI_OK;
}

// f / rec validation (pointers only; offsets are checked on the host only when
// the index arrays are host-visible, which device arrays are not)
adi_status check_src(const adi_source* f)
{
    if (!f || f->count == 0) return ADI_OK;
    if (f->count < 0 || f->count > ADI_MAX_SOURCES)
        return fail(ADI_EINVAL, "source count out of range [0, ADI_MAX_SOURCES]");
    if (!f->idx || !f->amp) return fail(ADI_EINVAL, "source idx/amp is null");
    return ADI_OK;
}

adi_status check_rec(const adi_receivers* r)
{
    if (!r || r->count == 0) return ADI_OK;
    if (r->count < 0) return fail(ADI_EINVAL, "negative receiver count");
    if (!r->idx || !r->traces) return fail(ADI_EINVAL, "receiver idx/traces is null");
    return ADI_OK;
}

template <typename T>
XArgs<T> make_x(const adi_wave_s* w, const void* u, const adi_source* f, int k, T rho_scale)
{
    XArgs<T> a{};
    a.u = static_cast<const T*>(u);
    a.r = static_cast<const T*>(w->r);
    a.qin = static_cast<const T*>(w->qin);
    a.w = static_cast<T*>(w->w);
    a.nx = w->nx;
    a.ny = w->ny;
    a.nseg = w->nseg;
    a.rows_per_strip = w->xp.fuse ? w->xp.frs : w->xp.rs;
    a.xcd = a.rows_per_strip <= kXcdStripRows;
    a.vec = ((size_t)w->nx * sizeof(T)) % 16 == 0 && aligned16(u) && aligned16(w->r) &&
            aligned16(w->w);
    a.sum = static_cast<T*>(w->sum);
    a.K = w->K;
    a.M = w->M;
    a.nxp = w->nxp;
    a.rho_scale = rho_scale;
    a.tau2 = (T)(w->dt * w->dt);
    if (f && f->count > 0) {
        a.nsrc = f->count;
        a.src_idx = f->idx;
        a.src_amp = static_cast<const T*>(f->amp) + (size_t)k * f->count;
    }
    a.nrec = w->tap_n;
    a.rec_idx = w->tap_idx;
    a.rec_out = static_cast<T*>(w->tap_out);
    return a;
}

template <typename T>
YArgs<T> make_y(const adi_wave_s* w, const void* u, const void* v, void* out, T alpha, T beta)
{
    YArgs<T> a{};
    a.w = static_cast<const T*>(w->w);
    a.r = static_cast<const T*>(w->r);
    a.nx = w->nx;
    a.ny = w->ny;
    a.M = w->M;
    a.K = w->K;
    a.nxp = w->nxp;
    a.tmp = static_cast<T*>(w->w);
    a.sum = static_cast<T*>(w->sum);
    a.X = static_cast<T*>(w->X);
    a.u = static_cast<const T*>(u);
    a.v = static_cast<const T*>(v);
    a.out = static_cast<T*>(out);
    a.alpha = alpha;
    a.beta = beta;
    return a;
}

int x_grid(const adi_wave_s* w)
{
    return xsweep_grid(w->ny, w->xp.fuse ? w->xp.frs : w->xp.rs, x_groups_per_wg(w->xp.tr));
}

// Queue one solve: x-sweep of `u` (with sources f at step k) then the y-chain
// writing out = alpha*u + beta*v + d.  `ev` (optional) receives 5 events
// bracketing the 4 launches.
template <typename T>
adi_status queue_solve(adi_wave_s* w, const void* u, const void* v, void* out, T alpha, T beta,
                       const adi_source* f, int k, T rho_scale, hipEvent_t* ev)
{
    hipStream_t st = w->stream;
    if (ev) ADI_HIP(hipEventRecord(ev[0], st));
    XArgs<T> xa = make_x<T>(w, u, f, k, rho_scale);
    if (!launch_x<T>(w->xp, x_grid(w), xa, st))
        return fail(ADI_EUNSUPPORTED, "no x-sweep kernel for this configuration");
    ADI_LAUNCHED("x_sweep_rhs");
    if (ev) ADI_HIP(hipEventRecord(ev[1], st));
    YArgs<T> ya = make_y<T>(w, u, v, out, alpha, beta);
    const dim3 yg((w->nx + 255) / 256, w->K);
    if (!w->xp.fuse) {
        hipLaunchKernelGGL((k_yreduce<T>), yg, dim3(256), 0, st, ya);
        ADI_LAUNCHED("y_reduce");
    }
    if (ev) ADI_HIP(hipEventRecord(ev[2], st));
    if (!launch_yscan<T>(w->yq, w->nx, ya, st))
        return fail(ADI_EUNSUPPORTED, "no y-interface kernel for this configuration");
    ADI_LAUNCHED("y_scan");
    if (ev) ADI_HIP(hipEventRecord(ev[3], st));
    if (!launch_ysolve<T>(w->M, yg, ya, st))
        return fail(ADI_EUNSUPPORTED, "no y-solve kernel for this chunk size");
    ADI_LAUNCHED("y_solve_update");
    if (ev) ADI_HIP(hipEventRecord(ev[4], st));
    return ADI_OK;
}

// The interface-system coefficients of the y-chunks depend on r only: built
// once (through the w buffer as scratch); every step then writes E and Pf.
template <typename T>
adi_status static_planes(adi_wave_s* w)
{
    YArgs<T> ya = make_y<T>(w, nullptr, nullptr, nullptr, T(0), T(0));
    const dim3 yg((w->nx + 255) / 256, w->K);
    hipLaunchKernelGGL((k_ystatic1<T>), yg, dim3(256), 0, w->stream, ya);
    ADI_LAUNCHED("y_static (pass 1)");
    hipLaunchKernelGGL((k_ystatic2<T>), yg, dim3(256), 0, w->stream, ya);
    ADI_LAUNCHED("y_static (pass 2)");
    return ADI_OK;
}

// One-pass step: the truncation error of a step is at most 4 qs^(K+1) max|w| (see
// fused.hpp); it is enabled only when that is below half an ulp of the arithmetic:
// 2^-24 for FP32 (K = 8), 2^-53 for FP64 (K = 16, the FP64 column strips).
bool fused_bound_holds(double rm, adi_dtype dt)
{
    if (!(rm >= 0.0) || !std::isfinite(rm)) return false;
    const double qs = rm > 0.0 ? (1.0 + 2.0 * rm - std::sqrt(1.0 + 4.0 * rm)) / (2.0 * rm) : 0.0;
    return dt == ADI_F64 ? 4.0 * std::pow(qs, FrCfg<double>::KY + 1) <= std::ldexp(1.0, -53)
                         : 4.0 * std::pow(qs, kFuKy + 1) <= std::ldexp(1.0, -24);
}

constexpr int kFuT8a = 16000, kFuT8b = 30;   // eight nodes per lane (fused.hpp)
constexpr int kFuT4a = 12000, kFuT4b = 15;   // four nodes per lane (fused4.hpp)
constexpr int kFuWmin = 64;

int fused_width(int nx, int ny, int ncu, int wmax, int ta, int tb, long long* cost)
{
    const int tx0 = (nx + wmax - 1) / wmax;
    auto width = [&](int tx) { return ((nx + tx - 1) / tx + 7) / 8 * 8; };
    int best = width(tx0);
    *cost = 0;
    if (ncu <= 0) return best;
    const long long ty = (ny + kFuHt - 1) / kFuHt;
    long long best_cost = -1;
    for (int tx = tx0; tx <= (nx + kFuWmin - 1) / kFuWmin; ++tx) {
        const int wt = width(tx);
        if (wt < kFuWmin && tx > tx0) break;
        const long long tiles = (long long)((nx + wt - 1) / wt) * ty;
        const long long rounds = (tiles + ncu - 1) / ncu;
        const long long c = rounds * (ta + (long long)tb * wt);
        if (best_cost < 0 || c < best_cost) {
            best_cost = c;
            best = wt;
        }
    }
    *cost = best_cost;
    return best;
}

// FP64 one-pass plan: column strips only (k_fusedr<double>), at most kFrS64 columns
// wide.  Set through adi_wave_set_tuning: one width (the given one, or the widest
// that covers nx evenly) and the given segment rows (else one segment per compute
// unit).  Otherwise the strip count from the fewest to twice as many whose largest
// segment has the least x-window work ((widest + 2 * 16 halo columns) * hs), with
// two widths 8 apart as for FP32.
void fused_plan_f64(adi_wave_s* w)
{
    constexpr int S = kFrS64, KX = FrCfg<double>::KX;
    const int ncu = w->f_ncu > 0 ? w->f_ncu : 1;
    const int nx = w->nx, ny = w->ny;
    int swt = w->f_wt_user > 0 ? std::min(w->f_wt_user, S) : 0, stx = 0, swide = 0, hs = w->f_hs_user > 0 ? w->f_hs_user : 0;
    if (swt > 0 || hs > 0) {
        if (swt == 0) {
            const int tx = (nx + S - 1) / S;
            swt = ((nx + tx - 1) / tx + 7) / 8 * 8;
        }
        stx = (nx + swt - 1) / swt;
        swide = stx;
        if (hs == 0) hs = (ny + std::max(1, ncu / stx) - 1) / std::max(1, ncu / stx);
    } else {
        long long best = -1;
        const int tx0 = (nx + S - 1) / S;
        for (int tx = tx0; tx <= 2 * tx0; ++tx) {
            const int w0 = nx / tx / 8 * 8;
            const int a = (nx - tx * w0 + 7) / 8;
            const int wmax = a > 0 ? w0 + 8 : w0;
            if (w0 < 8 || wmax > S || a > tx) continue;
            const int g = std::max(1, ncu / tx);
            const int h = (ny + g - 1) / g;
            const long long cost = (long long)(wmax + 2 * KX) * h;
            if (best < 0 || cost < best) {
                best = cost;
                swt = wmax; stx = tx; swide = a > 0 ? a : tx; hs = h;
            }
        }
        if (best < 0) {                      // narrower than 8 columns: one strip
            swt = (nx + 7) / 8 * 8; stx = 1; swide = 1; hs = ny;
        }
    }
    w->f_lane = FrCfg<double>::NPL;
    w->f_wt = swt;
    w->f_tx = stx;
    w->f_wide = swide;
    w->f_hs = hs;
    w->f_tiles = stx * ((ny + hs - 1) / hs);
    w->f_grid = (w->f_tiles + 7) / 8 * 8;
}

void fused_plan(adi_wave_s* w)
{
    const bool f64 = w->dtype == ADI_F64;
    w->fused_ok = ((f64 ? w->nx % 2 == 0 : w->nx % 4 == 0) && fused_bound_holds(w->rmax, w->dtype)) ? 1 : 0;
    const bool autoon = (long long)w->nx * w->ny >= (1LL << 16);
    w->fstep = w->fused_ok && (w->fused_mode == 1 || (w->fused_mode == 0 && autoon)) ? 1 : 0;
    if (f64) {
        fused_plan_f64(w);
        return;
    }
    long long c8 = 0, c4 = 0;
    const int w8 = fused_width(w->nx, w->ny, w->f_ncu, kFuWmax, kFuT8a, kFuT8b, &c8);
    const int w4 = fused_width(w->nx, w->ny, w->f_ncu, kF4Wmax, kFuT4a, kFuT4b, &c4);
    w->f_lane = w->f_lane_user ? w->f_lane_user : (w->f_ncu > 0 && c4 < c8) ? 4 : 8;
    const int wmax = w->f_lane == 4 ? kF4Wmax : kFuWmax;
    w->f_wt = w->f_wt_user > 0 ? std::min(w->f_wt_user, wmax) : (w->f_lane == 4 ? w4 : w8);
    w->f_tx = (w->nx + w->f_wt - 1) / w->f_wt;
    {
        long long c = 0;
        w->f4_wt = fused_width(w->nx, w->ny, 0, kF4Wmax, kFuT4a, kFuT4b, &c);
        w->f4_tx = (w->nx + w->f4_wt - 1) / w->f4_wt;
        w->f4_tiles = w->f4_tx * ((w->ny + kFuHt - 1) / kFuHt);
    }
    w->f_tiles = w->f_tx * ((w->ny + kFuHt - 1) / kFuHt);
    w->f_grid = (w->f_tiles + 7) / 8 * 8;
    w->f_wide = w->f_tx;
    // Column strips (fusedr.hpp): tx strips of two widths 8 apart (at most 240
    // columns) that cover nx, and g = ncu / tx segments of hs rows per strip, one per
    // compute unit.  Among the strip counts from the fewest, the one whose largest
    // segment has the least x-window work ((widest + 16 halo columns) * hs) is taken,
    // automatically when every segment then has at least kFrHmin rows (measured faster
    // than the tiles from 4096^2 to 8192^2); or set through adi_wave_set_tuning (one
    // width).
    w->f_hs = 0;
    long long c = 0;
    const int wt4 = fused_width(w->nx, w->ny, 0, kF4Wmax, kFuT4a, kFuT4b, &c);
    int hs = w->f_hs_user > 0 ? w->f_hs_user : 0;
    int swt = w->f_wt_user > 0 ? std::min(w->f_wt_user, kF4Wmax) : wt4;
    int stx = (w->nx + swt - 1) / swt, swide = stx;
    if (w->f_hs_user == 0 && w->f_ncu > 0 && w->f_wt_user == 0 && w->f_lane_user == 0) {
        long long best = -1;
        for (int tx = (w->nx + kF4Wmax - 1) / kF4Wmax; tx <= (w->nx + kF4Wmax - 1) / kF4Wmax + 4; ++tx) {
            const int w0 = w->nx / tx / 8 * 8;
            const int a = (w->nx - tx * w0 + 7) / 8;           // strips one width step wider
            const int wmax = a > 0 ? w0 + 8 : w0;
            const int g = w->f_ncu / tx;
            if (w0 < 8 || wmax > kF4Wmax || a > tx || g <= 0) continue;
            const int h = (w->ny + g - 1) / g;
            if (h < kFrHmin) continue;
            const long long cost = (long long)(wmax + 2 * kFuKx) * h;
            if (best < 0 || cost < best) {
                best = cost;
                hs = h;
                swt = wmax;
                stx = tx;
                swide = a > 0 ? a : tx;
            }
        }
    }
    if (hs > 0) {
        w->f_lane = 4;
        w->f_wt = swt;
        w->f_tx = stx;
        w->f_wide = swide;
        w->f_hs = hs;
        w->f_tiles = w->f_tx * ((w->ny + hs - 1) / hs);
        w->f_grid = (w->f_tiles + 7) / 8 * 8;   // a multiple of 8 for the XCD-aware block map
    }
}

// largest r of an FP32 handle (synchronises the stream); X is free scratch here
template <typename T>
adi_status measure_rmax(adi_wave_s* w)
{
    const long long n = (long long)w->nx * w->ny;
    ADI_HIP(hipMemsetAsync(w->X, 0, sizeof(T), w->stream));   // X holds at least one value
    const int grid = (int)std::min<long long>((n + 255) / 256, 2048);
    if constexpr (sizeof(T) == 4) {
        hipLaunchKernelGGL(k_rmax, dim3(grid), dim3(256), 0, w->stream, static_cast<const float*>(w->r), n,
                           static_cast<unsigned int*>(w->X));
    } else {
        hipLaunchKernelGGL(k_rmax64, dim3(grid), dim3(256), 0, w->stream, static_cast<const double*>(w->r), n,
                           static_cast<unsigned long long*>(w->X));
    }
    ADI_LAUNCHED("rmax");
    T v = T(0);
    ADI_HIP(hipMemcpyAsync(&v, w->X, sizeof(T), hipMemcpyDeviceToHost, w->stream));
    ADI_HIP(hipStreamSynchronize(w->stream));
    w->rmax = (double)v;
    fused_plan(w);
    return ADI_OK;
}

void adjoint_invalidate(adi_wave_s* w);   // adjoint.hpp

template <typename T>
adi_status set_coef(adi_wave_s* w, const void* field, double scalar, int squared, bool measure = true)
{
    ++w->gen;
    adjoint_invalidate(w);   // a stored forward record no longer matches the coefficient
    const long long n = (long long)w->nx * w->ny;
    const double s = w->dt * w->dt / (2.0 * w->h * w->h);
    const int grid = (int)std::min<long long>((n + 255) / 256, 65536);
    hipLaunchKernelGGL((k_coef<T>), dim3(grid), dim3(256), 0, w->stream,
                       static_cast<const T*>(field), (T)scalar, squared, (T)s,
                       static_cast<T*>(w->r), n);
    ADI_LAUNCHED("coef");
    hipLaunchKernelGGL((k_xpivots<T>), dim3((w->ny + 255) / 256), dim3(256), 0, w->stream,
                       static_cast<const T*>(w->r), static_cast<T*>(w->qin), w->nx, w->ny, w->nseg);
    ADI_LAUNCHED("x_pivots");
    if (w->qin2) {
        hipLaunchKernelGGL((k_xpivots<T, 2>), dim3((w->ny + 255) / 256), dim3(256), 0, w->stream,
                           static_cast<const T*>(w->r), static_cast<T*>(w->qin2), w->nx, w->ny, (w->nx + 1) / 2);
        ADI_LAUNCHED("x_pivots (2-node lanes)");
    }
    if (measure)
        if (adi_status s = measure_rmax<T>(w)) return s;
    return static_planes<T>(w);
}

template <typename T>
FArgsT<T> make_fargs(const adi_wave_s* w, const void* u_curr, void* u_prev, const adi_source* f, int k)
{
    FArgsT<T> a{};
    a.uc = static_cast<const T*>(u_curr);
    a.up = static_cast<T*>(u_prev);
    a.r = static_cast<const T*>(w->r);
    a.qin = static_cast<const T*>(w->qin);
    a.nx = w->nx;
    a.ny = w->ny;
    a.nseg = w->nseg;
    a.wt = w->f_wt;
    a.tiles_x = w->f_tx;
    a.wide = w->f_wide;
    a.tiles = w->f_tiles;
    a.xcd_map = 1;
    a.tau2 = (T)(w->dt * w->dt);
    if (f && f->count > 0) {
        a.nsrc = f->count;
        a.src_idx = f->idx;
        a.src_amp = static_cast<const T*>(f->amp) + (size_t)k * f->count;
    }
    a.nrec = w->tap_n;
    a.rec_idx = w->tap_idx;
    a.rec_out = static_cast<T*>(w->tap_out);
    a.hs = w->f_hs;
    return a;
}

adi_status queue_fused(adi_wave_s* w, const void* u_curr, void* u_prev, const adi_source* f, int k)
{
    if (w->dtype == ADI_F64) {
        FArgsT<double> a = make_fargs<double>(w, u_curr, u_prev, f, k);
        a.qin = static_cast<const double*>(w->qin2);   // entry pivot of every 2-node lane
        hipLaunchKernelGGL(k_fusedr<double>, dim3(w->f_grid), dim3(kFrThreads64), 0, w->stream, a);
        ADI_LAUNCHED("fused_step");
        return ADI_OK;
    }
    const FArgs a = make_fargs<float>(w, u_curr, u_prev, f, k);
    if (w->f_hs > 0)
        hipLaunchKernelGGL(k_fusedr<float>, dim3(w->f_grid), dim3(kFrThreads), 0, w->stream, a);
    else if (w->f_lane == 4)
        hipLaunchKernelGGL(k_fused4, dim3(w->f_grid), dim3(1024), 0, w->stream, a);
    else
        hipLaunchKernelGGL(k_fused, dim3(w->f_grid), dim3(1024), 0, w->stream, a);
    ADI_LAUNCHED("fused_step");
    return ADI_OK;
}

int cr_levels(int n)   // m with 2^m - 1 >= n
{
    int m = 1;
    while ((1LL << m) - 1 < n) ++m;
    return m;
}

int cr_grid(long long work) { return (int)std::max<long long>(1, std::min<long long>((work + 255) / 256, 1 << 16)); }

// all lines of one sweep by cyclic reduction, one launch per level (d holds the
// right-hand sides and receives the solutions)
template <typename T>
adi_status queue_cr_lines(adi_wave_s* w, CrArgs<T> A)
{
    const int m = cr_levels(A.n);
    for (int k = 1; k < m; ++k) {
        A.h = 1 << (k - 1);
        hipLaunchKernelGGL((k_cr_forward<T>), dim3(cr_grid((long long)(A.n / (2 * A.h)) * A.lines)), dim3(256), 0,
                           w->stream, A);
        ADI_LAUNCHED("cr_forward");
    }
    A.h = 1 << (m - 1);
    hipLaunchKernelGGL((k_cr_div<T>), dim3(cr_grid(A.lines)), dim3(256), 0, w->stream, A);
    ADI_LAUNCHED("cr_div");
    for (int k = m - 1; k >= 1; --k) {
        A.h = 1 << (k - 1);
        hipLaunchKernelGGL((k_cr_backward<T>), dim3(cr_grid((long long)((A.n / A.h + 1) / 2) * A.lines)), dim3(256),
                           0, w->stream, A);
        ADI_LAUNCHED("cr_backward");
    }
    return ADI_OK;
}

// one ADI step with cyclic-reduction line solves: out = alpha u + beta v + d
template <typename T>
adi_status queue_cr_step(adi_wave_s* w, const void* u, const void* v, void* out, T alpha, T beta,
                         const adi_source* f, int k, T rho_scale)
{
    const long long n = (long long)w->nx * w->ny;
    T* a = static_cast<T*>(w->cr_abc);
    T* b = a + n;
    T* c = b + n;
    T* d = static_cast<T*>(w->w);
    const T* r = static_cast<const T*>(w->r);
    hipLaunchKernelGGL((k_cr_setup<T>), dim3(cr_grid(n)), dim3(256), 0, w->stream, static_cast<const T*>(u), r, a,
                       b, c, d, w->nx, w->ny, 0, rho_scale);
    ADI_LAUNCHED("cr_setup_x");
    if (f && f->count > 0) {
        hipLaunchKernelGGL((k_cr_sources<T>), dim3(1), dim3(64), 0, w->stream, d, f->idx,
                           static_cast<const T*>(f->amp) + (size_t)k * f->count, f->count,
                           (T)(rho_scale * (T)(w->dt * w->dt)), n);
        ADI_LAUNCHED("cr_sources");
    }
    CrArgs<T> X{a, b, c, d, w->nx, w->ny, (long long)w->nx, 1LL, 0};
    if (adi_status s = queue_cr_lines<T>(w, X)) return s;
    hipLaunchKernelGGL((k_cr_setup<T>), dim3(cr_grid(n)), dim3(256), 0, w->stream, static_cast<const T*>(u), r, a,
                       b, c, d, w->nx, w->ny, 1, rho_scale);
    ADI_LAUNCHED("cr_setup_y");
    CrArgs<T> Y{a, b, c, d, w->ny, w->nx, 1LL, (long long)w->nx, 0};
    if (adi_status s = queue_cr_lines<T>(w, Y)) return s;
    hipLaunchKernelGGL((k_cr_update<T>), dim3(cr_grid(n)), dim3(256), 0, w->stream, static_cast<const T*>(u),
                       static_cast<const T*>(v), d, static_cast<T*>(out), alpha, beta, n);
    ADI_LAUNCHED("cr_update");
    return ADI_OK;
}

// kind: kStepDefault = the handle's step (cyclic reduction when asked for, else the
// one-pass step when allowed, else the exact two-pass step); kStepNoCr = the same
// without cyclic reduction; kStepExact = the exact two-pass step
enum { kStepDefault = 0, kStepNoCr = 1, kStepExact = 2 };

template <typename T>
adi_status do_step(adi_wave_s* w, void** u_prev, void** u_curr, const adi_source* f,
                   const adi_receivers* rec, int nsteps, int kind = kStepDefault)
{
    const bool cr = kind == kStepDefault && w->cr;
    const bool fused = !cr && kind != kStepExact && w->fstep && aligned16(*u_prev) && aligned16(*u_curr);
    const bool recs = rec && rec->count > 0;
    auto record = [&](int k, const void* level) -> adi_status {
        hipLaunchKernelGGL((k_record<T>), dim3((rec->count + 255) / 256), dim3(256), 0, w->stream,
                           static_cast<const T*>(level), rec->idx,
                           static_cast<T*>(rec->traces) + (size_t)k * rec->count, rec->count,
                           (long long)w->nx * w->ny);
        ADI_LAUNCHED("record");
        return ADI_OK;
    };
    for (int k = 0; k < nsteps; ++k) {
        // the x-sweep and one-pass launches record the previous step's receivers
        if (recs && !cr && k > 0) {
            w->tap_n = rec->count;
            w->tap_idx = rec->idx;
            w->tap_out = static_cast<T*>(rec->traces) + (size_t)(k - 1) * rec->count;
        }
        adi_status s = cr      ? queue_cr_step<T>(w, *u_curr, *u_prev, *u_prev, T(2), T(-1), f, k, T(1))
                       : fused ? queue_fused(w, *u_curr, *u_prev, f, k)
                               : queue_solve<T>(w, *u_curr, *u_prev, *u_prev, T(2), T(-1), f, k, T(1), nullptr);
        w->tap_n = 0;
        w->tap_idx = nullptr;
        w->tap_out = nullptr;
        if (s != ADI_OK) return s;
        if (recs && cr)
            if (adi_status s2 = record(k, *u_prev)) return s2;
        std::swap(*u_prev, *u_curr);
    }
    if (recs && !cr && nsteps > 0) return record(nsteps - 1, *u_curr);
    return ADI_OK;
}

template <typename T>
adi_status do_start(adi_wave_s* w, const void* u0, const void* psi, const adi_source* f0, int mode,
                    void* u1)
{
    if (mode == ADI_START_PAPER) {
        const long long n = (long long)w->nx * w->ny;
        const int grid = (int)std::min<long long>((n + 255) / 256, 65536);
        hipLaunchKernelGGL((k_start_paper<T>), dim3(grid), dim3(256), 0, w->stream,
                           static_cast<const T*>(u0), static_cast<const T*>(psi), (T)w->dt,
                           static_cast<T*>(u1), n);
        ADI_LAUNCHED("start_paper");
        return ADI_OK;
    }
    // ghost start: u1 = u0 + dt psi + e,  (I - bKLxx)(I - bKLyy) e = rho(u0, f0) / 2
    return queue_solve<T>(w, u0, psi, u1, T(1), psi ? (T)w->dt : T(0), f0, 0, T(0.5), nullptr);
}

}  // namespace

// ================================================================== C ABI ====
extern "C" {

const char* adi_last_error(void) { return g_err.c_str(); }

adi_status adi_wave_create(adi_wave_t* out, int nx, int ny, double h, double dt, const void* speed,
                           double speed_scalar, adi_dtype dtype, void* hip_stream)
{
    if (!out) return fail(ADI_EINVAL, "out is null");
    *out = nullptr;
    if (dtype != ADI_F32 && dtype != ADI_F64) return fail(ADI_EINVAL, "unknown dtype");
    if (nx < 1 || ny < 1) return fail(ADI_EINVAL, "nx and ny must be >= 1");
    if ((long long)nx * ny >= (1LL << 31)) return fail(ADI_EUNSUPPORTED, "nx*ny must be < 2^31");
    if (ny > 16384) return fail(ADI_EUNSUPPORTED, "ny > 16384 is not supported");
    if (!finite_pos(h) || !finite_pos(dt)) return fail(ADI_EINVAL, "h and dt must be finite and > 0");
    if (!speed && !finite_pos(speed_scalar))
        return fail(ADI_EINVAL, "speed_scalar must be finite and > 0 when speed is NULL");
    XPlan xp{};
    if (!choose_x(nx, dtype, xp))
        return fail(ADI_EUNSUPPORTED, "nx > 8192 is not supported");
    xp.rs = choose_rows(ny, xp.tr);
    // chunk rows: 32 unless the y-solve would have fewer than 512 workgroups
    int M = ((long long)((nx + 255) / 256) * ((ny + 31) / 32) >= 512) ? 32 : 16;
    // fusing the y-chunk reduction into the x-sweep needs a strip per workgroup
    // on every CU; fused strips are whole chunks: (chunk rows, strip rows) from
    // (32, 32), (16, 32), (16, 16), the first that gives enough strips
    xp.fuse = 0;
    xp.frs = fused_rows(M);
    if (fuse_fits(xp.tr, dtype)) {
        static const int cand[][2] = {{32, 32}, {16, 32}, {16, 16}};
        for (auto& c : cand) {
            if (c[0] > M) continue;
            const long long wgs = ((ny + c[1] - 1) / c[1] + x_groups_per_wg(xp.tr) - 1) / x_groups_per_wg(xp.tr);
            if (wgs >= 256) { M = c[0]; xp.frs = c[1]; xp.fuse = 1; break; }
        }
    }

    adi_wave_s* w = new adi_wave_s();
    w->nx = nx; w->ny = ny; w->h = h; w->dt = dt; w->dtype = dtype;
    w->stream = static_cast<hipStream_t>(hip_stream);
    w->xp = xp;
    w->M = M;
    if (hipGetDevice(&w->device) != hipSuccess) {
        delete w;
        return fail(ADI_EHIP, "hipGetDevice failed");
    }
    if (hipDeviceGetAttribute(&w->f_ncu, hipDeviceAttributeMultiprocessorCount, w->device) != hipSuccess) {
        (void)hipGetLastError();
        w->f_ncu = 0;
    }
    const size_t es = esize(dtype);
    const size_t npts = (size_t)nx * ny;
    w->nseg = (nx + kSeg - 1) / kSeg;
    if (hipMalloc(&w->r, npts * es) != hipSuccess ||
        hipMalloc(&w->qin, (size_t)ny * w->nseg * es) != hipSuccess ||
        (dtype == ADI_F64 && hipMalloc(&w->qin2, (size_t)ny * ((nx + 1) / 2) * es) != hipSuccess)) {
        (void)hipGetLastError();
        free_ws(w);
        delete w;
        return fail(ADI_ENOMEM, "hipMalloc of the coefficient/x-sweep fields failed");
    }
    adi_status s = alloc_chunks(w);
    if (s == ADI_OK)
        s = (dtype == ADI_F32) ? set_coef<float>(w, speed, speed_scalar, 1)
                               : set_coef<double>(w, speed, speed_scalar, 1);
    if (s == ADI_OK && hipStreamSynchronize(w->stream) != hipSuccess)
        s = fail(ADI_EHIP, "stream synchronise after create failed");
    if (s != ADI_OK) {
        free_ws(w);
        delete w;
        return s;
    }
    *out = w;
    return ADI_OK;
}

adi_status adi_wave_set_kappa(adi_wave_t w, const void* kappa, double kappa_scalar)
{
    if (adi_status s = check_handle(w)) return s;
    if (!kappa && !finite_pos(kappa_scalar))
        return fail(ADI_EINVAL, "kappa_scalar must be finite and > 0 when kappa is NULL");
    return w->dtype == ADI_F32 ? set_coef<float>(w, kappa, kappa_scalar, 0)
                               : set_coef<double>(w, kappa, kappa_scalar, 0);
}

adi_status adi_wave_set_stream(adi_wave_t w, void* hip_stream)
{
    if (adi_status s = check_handle(w)) return s;
    w->stream = static_cast<hipStream_t>(hip_stream);
    return ADI_OK;
}

adi_status adi_wave_start(adi_wave_t w, const void* u0, const void* psi, const adi_source* f0,
                          int mode, void* u1)
{
    if (adi_status s = check_handle(w)) return s;
    if (!u0 || !u1) return fail(ADI_EINVAL, "u0 and u1 must be non-null");
    if (u1 == u0 || (psi && u1 == psi)) return fail(ADI_EINVAL, "u1 must not alias u0 or psi");
    if (mode != ADI_START_PAPER && mode != ADI_START_GHOST) return fail(ADI_EINVAL, "unknown start mode");
    if (adi_status s = check_src(f0)) return s;
    return w->dtype == ADI_F32 ? do_start<float>(w, u0, psi, f0, mode, u1)
                               : do_start<double>(w, u0, psi, f0, mode, u1);
}

adi_status adi_wave_step(adi_wave_t w, void** u_prev, void** u_curr, const adi_source* f,
                         const adi_receivers* rec, int nsteps)
{
    if (adi_status s = check_handle(w)) return s;
    if (!u_prev || !u_curr || !*u_prev || !*u_curr) return fail(ADI_EINVAL, "null level pointer");
    if (*u_prev == *u_curr) return fail(ADI_EINVAL, "u_prev and u_curr must be distinct buffers");
    if (nsteps < 0) return fail(ADI_EINVAL, "nsteps must be >= 0");
    if (adi_status s = check_src(f)) return s;
    if (adi_status s = check_rec(rec)) return s;
    return w->dtype == ADI_F32 ? do_step<float>(w, u_prev, u_curr, f, rec, nsteps)
                               : do_step<double>(w, u_prev, u_curr, f, rec, nsteps);
}

adi_status adi_wave_destroy(adi_wave_t w)
{
    if (!w) return ADI_OK;
    (void)hipStreamSynchronize(w->stream);
    free_ws(w);
    adjoint_free(w->adj);
    delete w;
    return ADI_OK;
}

adi_status adi_wave_get_info(adi_wave_t w, adi_wave_info* info)
{
    if (adi_status s = check_handle(w)) return s;
    if (!info) return fail(ADI_EINVAL, "info is null");
    info->nx = w->nx;
    info->ny = w->ny;
    info->dtype = (int)w->dtype;
    info->x_threads_per_line = w->xp.tr;
    info->x_rows_per_strip = w->xp.fuse ? w->xp.frs : w->xp.rs;
    info->y_fused = w->xp.fuse;
    info->y_chunk_rows = w->M;
    info->y_chunks = w->K;
    info->kernels_per_step = w->cr ? 1 + 2 * cr_levels(w->nx) + 2 * cr_levels(w->ny)
                                   : w->fstep ? 1 : (w->xp.fuse ? 3 : 4);
    info->workspace_bytes = w->bytes;
    info->fused_step = w->fstep;
    info->fused_allowed = w->fused_ok;
    info->r_max = w->rmax;
    info->line_solver = w->cr ? 2 : 1;
    info->fused_tile_cols = w->f_wt;
    info->fused_tiles = w->f_tiles;
    info->fused_lane_nodes = w->f_lane;
    info->fused_segment_rows = w->f_hs;
    info->fused_strips_wide = w->f_wide;
    return ADI_OK;
}

adi_status adi_wave_set_tuning(adi_wave_t w, const adi_tuning* t)
{
    if (adi_status s = check_handle(w)) return s;
    if (!t) return fail(ADI_EINVAL, "tuning is null");
    XPlan xp = w->xp;
    if (t->x_threads_per_line > 0) xp.tr = t->x_threads_per_line;
    if (t->x_rows_per_strip > 0) xp.rs = t->x_rows_per_strip;
    if (t->y_fused == 1) xp.fuse = 1;
    if (t->y_fused == 2) xp.fuse = 0;
    if (xp.tr != 64 && xp.tr != 128 && xp.tr != 256 && xp.tr != 1024)
        return fail(ADI_EINVAL, "x_threads_per_line must be 64, 128, 256 or 1024");
    if (8LL * xp.tr < w->nx) return fail(ADI_EINVAL, "8 * x_threads_per_line must cover nx");
    if (xp.fuse && !fuse_fits(xp.tr, w->dtype))
        return fail(ADI_EUNSUPPORTED, "fused y-reduction does not fit in LDS for this plan");
    const int M = t->y_chunk_rows > 0 ? t->y_chunk_rows : w->M;
    if (M != 16 && M != 32) return fail(ADI_EINVAL, "y_chunk_rows must be 16 or 32");
    if (t->fused_step < 0 || t->fused_step > 2) return fail(ADI_EINVAL, "fused_step must be 0, 1 or 2");
    if (t->fused_step == 1 && !w->fused_ok)
        return fail(ADI_EUNSUPPORTED, w->dtype == ADI_F64
                                          ? "the FP64 one-pass step needs nx % 2 == 0 and r <= 0.13 everywhere"
                                          : "the one-pass step needs nx % 4 == 0 and r <= 0.18 everywhere");
    if (w->dtype == ADI_F64) {
        // FP64 runs on column strips only, at most kFrS64 columns wide
        if (t->fused_lane_nodes > 0 || t->fused_segment_rows == -2)
            return fail(ADI_EINVAL, "the FP64 one-pass step runs on column strips (no tiles, no lane setting)");
        if (t->fused_tile_cols > 0 && (t->fused_tile_cols % 8 != 0 || t->fused_tile_cols > kFrS64))
            return fail(ADI_EINVAL, "FP64 column strips: fused_tile_cols must be a multiple of 8 and at most 64");
    }
    if (t->fused_lane_nodes != 0 && t->fused_lane_nodes != -1 && t->fused_lane_nodes != 4 &&
        t->fused_lane_nodes != 8)
        return fail(ADI_EINVAL, "fused_lane_nodes must be -1, 0, 4 or 8");
    const int lane_nodes = t->fused_lane_nodes > 0 ? t->fused_lane_nodes : w->f_lane;
    const int wmax = lane_nodes == 4 ? kF4Wmax : kFuWmax;
    const int wt_req = t->fused_tile_cols > 0 ? t->fused_tile_cols : 0;
    if (wt_req > 0 && (wt_req % 8 != 0 || wt_req > wmax))
        return fail(ADI_EINVAL, "fused_tile_cols must be a multiple of 8 and at most 496 (240 with 4 nodes per lane)");
    if (t->fused_segment_rows < -2 || (t->fused_segment_rows > 0 && t->fused_segment_rows < 8))
        return fail(ADI_EINVAL, "fused_segment_rows must be -2, -1, 0 or at least 8");
    if (t->fused_segment_rows > 0 && t->fused_lane_nodes == 8)
        return fail(ADI_EINVAL, "column strips take four nodes per lane");
    if (t->fused_segment_rows > 0 && wt_req > kF4Wmax)
        return fail(ADI_EINVAL, "column strips are at most 240 columns wide");
    if (t->fused_step > 0) w->fused_mode = t->fused_step;
    if (t->fused_segment_rows) w->f_hs_user = t->fused_segment_rows == -1 ? 0 : t->fused_segment_rows;
    if (t->fused_tile_cols > 0) w->f_wt_user = t->fused_tile_cols;
    if (t->fused_tile_cols == -1) w->f_wt_user = 0;
    if (t->fused_lane_nodes) w->f_lane_user = t->fused_lane_nodes > 0 ? t->fused_lane_nodes : 0;
    if (t->fused_step > 0 || t->fused_tile_cols > 0 || t->fused_tile_cols == -1 || t->fused_lane_nodes ||
        t->fused_segment_rows)
        fused_plan(w);
    if (t->line_solver < 0 || t->line_solver > 2) return fail(ADI_EINVAL, "line_solver must be 0, 1 or 2");
    if (t->line_solver == 2 && !w->cr_abc) {
        const size_t bytes = 3 * (size_t)w->nx * w->ny * esize(w->dtype);
        if (hipMalloc(&w->cr_abc, bytes) != hipSuccess) {
            (void)hipGetLastError();
            w->cr_abc = nullptr;
            return fail(ADI_ENOMEM, "hipMalloc of the cyclic-reduction coefficients failed");
        }
        w->bytes += bytes;
    }
    if (t->line_solver > 0) w->cr = t->line_solver == 2 ? 1 : 0;
    if (xp.fuse && (M != w->M || !w->xp.fuse)) xp.frs = fused_rows(M);
    w->xp = xp;
    if (M != w->M) {
        if (hipStreamSynchronize(w->stream) != hipSuccess)
            return fail(ADI_EHIP, "stream synchronise failed");
        w->M = M;
        if (adi_status s = alloc_chunks(w)) return s;
        return w->dtype == ADI_F32 ? static_planes<float>(w) : static_planes<double>(w);
    }
    return ADI_OK;
}

adi_status adi_wave_profile(adi_wave_t w, void** u_prev, void** u_curr, const adi_source* f,
                            int nsteps, double* ms_per_kernel, const char** names, int* nkinds)
{
    if (adi_status s = check_handle(w)) return s;
    if (!u_prev || !u_curr || !*u_prev || !*u_curr) return fail(ADI_EINVAL, "null level pointer");
    if (*u_prev == *u_curr) return fail(ADI_EINVAL, "u_prev and u_curr must be distinct buffers");
    if (nsteps < 1 || nsteps > 100000) return fail(ADI_EINVAL, "nsteps must be in [1, 100000]");
    if (!ms_per_kernel || !nkinds) return fail(ADI_EINVAL, "null output");
    if (adi_status s = check_src(f)) return s;
    static const char* kNames[4] = {"x_sweep_rhs", "y_reduce", "y_scan", "y_solve_update"};
    std::vector<hipEvent_t> ev((size_t)nsteps * 5, nullptr);
    adi_status st = ADI_OK;
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) { st = fail(ADI_EHIP, "hipEventCreate failed"); break; }
    const bool cr = w->cr != 0;
    const bool fused = cr || (w->fstep && aligned16(*u_prev) && aligned16(*u_curr));
    for (int k = 0; k < nsteps && st == ADI_OK; ++k) {
        hipEvent_t* e = &ev[(size_t)k * 5];
        if (fused) {   // one timed range per step (one-pass step, or the whole cyclic-reduction step)
            if (hipEventRecord(e[0], w->stream) != hipSuccess) st = fail(ADI_EHIP, "hipEventRecord failed");
            if (st == ADI_OK)
                st = !cr ? queue_fused(w, *u_curr, *u_prev, f, k)
                   : w->dtype == ADI_F32
                       ? queue_cr_step<float>(w, *u_curr, *u_prev, *u_prev, 2.f, -1.f, f, k, 1.f)
                       : queue_cr_step<double>(w, *u_curr, *u_prev, *u_prev, 2.0, -1.0, f, k, 1.0);
            if (st == ADI_OK && hipEventRecord(e[1], w->stream) != hipSuccess)
                st = fail(ADI_EHIP, "hipEventRecord failed");
        } else {
            st = w->dtype == ADI_F32
                     ? queue_solve<float>(w, *u_curr, *u_prev, *u_prev, 2.f, -1.f, f, k, 1.f, e)
                     : queue_solve<double>(w, *u_curr, *u_prev, *u_prev, 2.0, -1.0, f, k, 1.0, e);
        }
        if (st == ADI_OK) std::swap(*u_prev, *u_curr);
    }
    if (st == ADI_OK && hipStreamSynchronize(w->stream) != hipSuccess)
        st = fail(ADI_EHIP, "stream synchronise failed");
    if (st == ADI_OK && fused) {
        double acc = 0.0;
        for (int k = 0; k < nsteps && st == ADI_OK; ++k) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[(size_t)k * 5], ev[(size_t)k * 5 + 1]) != hipSuccess)
                st = fail(ADI_EHIP, "hipEventElapsedTime failed");
            acc += ms;
        }
        if (st == ADI_OK) {
            ms_per_kernel[0] = acc / nsteps;
            if (names) names[0] = cr ? "cr_step" : "fused_step";
            *nkinds = 1;
        }
    } else if (st == ADI_OK) {
        double acc[4] = {0, 0, 0, 0};
        for (int k = 0; k < nsteps && st == ADI_OK; ++k)
            for (int q = 0; q < 4; ++q) {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, ev[(size_t)k * 5 + q], ev[(size_t)k * 5 + q + 1]) != hipSuccess) {
                    st = fail(ADI_EHIP, "hipEventElapsedTime failed");
                    break;
                }
                acc[q] += ms;
            }
        if (st == ADI_OK) {
            // a fused plan has no separate y_reduce launch: its x-sweep does that work
            static const char* kFusedX = "x_sweep_rhs_y_reduce";
            int n = 0;
            for (int q = 0; q < 4; ++q) {
                if (q == 1 && w->xp.fuse) continue;
                ms_per_kernel[n] = acc[q] / nsteps;
                if (names) names[n] = (q == 0 && w->xp.fuse) ? kFusedX : kNames[q];
                ++n;
            }
            *nkinds = n;
        }
    }
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    return st;
}

adi_status adi_stream_copy(const void* src, void* dst, size_t bytes, void* hip_stream)
{
    if (!src || !dst) return fail(ADI_EINVAL, "null pointer");
    if (bytes % 16 != 0 || !aligned16(src) || !aligned16(dst))
        return fail(ADI_EINVAL, "bytes must be a multiple of 16 and pointers 16-byte aligned");
    const long long n = (long long)(bytes / 16);
    if (n == 0) return ADI_OK;
    const int grid = (int)std::min<long long>((n + 255) / 256, 1 << 20);
    hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                       static_cast<const float4*>(src), static_cast<float4*>(dst), n);
    ADI_LAUNCHED("copy");
    return ADI_OK;
}

}  // extern "C"

namespace {

// Argument checks shared by the two batched-solve entry points.  On success *wg
// tells whether the on-chip one-workgroup-per-system kernels take the layout
// (with plan *p), else the partition solve does (it needs a workspace).
adi_status tri_check(adi_dtype dtype, int n, int batch, const void* a, const void* b, const void* c,
                     const void* d, long long sys_stride, long long elem_stride, bool* wg, TPlan* p)
{
    if (dtype != ADI_F32 && dtype != ADI_F64) return fail(ADI_EINVAL, "unknown dtype");
    if (n < 0 || batch < 0) return fail(ADI_EINVAL, "n and batch must be >= 0");
    *wg = false;
    if (n == 0 || batch == 0) return ADI_OK;
    if (!a || !b || !c || !d) return fail(ADI_EINVAL, "null array");
    if (d == a || d == b || d == c) return fail(ADI_EINVAL, "d must not alias a, b or c");
    if (elem_stride < 1) return fail(ADI_EINVAL, "elem_stride must be >= 1");
    if (batch > 1 && sys_stride < 1) return fail(ADI_EINVAL, "sys_stride must be >= 1 when batch > 1");
    *wg = elem_stride == 1 && choose_tri(n, dtype, *p);
    return ADI_OK;
}

adi_status tri_run_wg(adi_dtype dtype, const TPlan& p, int n, int batch, const void* a, const void* b,
                      const void* c, void* d, long long sys_stride, long long elem_stride, hipStream_t st)
{
    const size_t es = esize(dtype);
    const bool vec = aligned16(a) && aligned16(b) && aligned16(c) && aligned16(d) &&
                     ((size_t)sys_stride * es) % 16 == 0 && ((size_t)p.s * es) % 16 == 0;
    bool ok;
    if (dtype == ADI_F32) {
        TriArgs<float> t{(const float*)a, (const float*)b, (const float*)c, (float*)d, n, batch,
                         sys_stride, elem_stride, vec};
        ok = launch_tri<float>(p, batch, t, st);
    } else {
        TriArgs<double> t{(const double*)a, (const double*)b, (const double*)c, (double*)d, n, batch,
                          sys_stride, elem_stride, vec};
        ok = launch_tri<double>(p, batch, t, st);
    }
    if (!ok) return fail(ADI_EUNSUPPORTED, "no batched kernel for this size");
    ADI_LAUNCHED("tridiag_wg");
    return ADI_OK;
}

size_t tri_part_bytes(adi_dtype dtype, int n, int batch)
{
    return (dtype == ADI_F32 ? tri_part_workspace<float>(n, batch) : tri_part_workspace<double>(n, batch)) *
           esize(dtype);
}

adi_status tri_run_part(adi_dtype dtype, int n, int batch, const void* a, const void* b, const void* c, void* d,
                        long long sys_stride, long long elem_stride, void* scr, hipStream_t st)
{
    if (dtype == ADI_F32) {
        TriArgs<float> t{(const float*)a, (const float*)b, (const float*)c, (float*)d, n, batch,
                         sys_stride, elem_stride, 0};
        launch_tri_part<float>(t, (float*)scr, st);
    } else {
        TriArgs<double> t{(const double*)a, (const double*)b, (const double*)c, (double*)d, n, batch,
                          sys_stride, elem_stride, 0};
        launch_tri_part<double>(t, (double*)scr, st);
    }
    ADI_LAUNCHED("tridiag_part");
    return ADI_OK;
}

// scratch of the partition solve, one per device, grown on demand
std::mutex g_scr_mu;
std::vector<std::pair<void*, size_t>> g_scr;

// The allocation-free variant's scratch: a fixed array in the library's code
// object, one copy per device.  In host code `scratch` names a host-side
// stand-in, so the kernels get the device address that hipGetSymbolAddress
// returns for the current device, looked up once per device and kept.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
std::mutex g_na_mu;
std::vector<void*> g_na_ptr;

adi_status noalloc_scratch(void** out)
{
    int dev = 0;
    ADI_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_na_mu);
    if ((int)g_na_ptr.size() <= dev) g_na_ptr.resize(dev + 1, nullptr);
    if (!g_na_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(ADI_EHIP, std::string("hipGetSymbolAddress of the no-allocation scratch: ") +
                                      hipGetErrorString(e));
        g_na_ptr[dev] = ptr;
    }
    *out = g_na_ptr[dev];
    return ADI_OK;
}

}  // namespace

extern "C" {

adi_status tridiag_solve_batched(adi_dtype dtype, int n, int batch, const void* a, const void* b,
                                 const void* c, void* d, long long sys_stride,
                                 long long elem_stride, void* hip_stream)
{
    bool wg = false;
    TPlan p{};
    if (adi_status s = tri_check(dtype, n, batch, a, b, c, d, sys_stride, elem_stride, &wg, &p)) return s;
    if (n == 0 || batch == 0) return ADI_OK;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (wg) return tri_run_wg(dtype, p, n, batch, a, b, c, d, sys_stride, elem_stride, st);
    int dev = 0;
    ADI_HIP(hipGetDevice(&dev));
    const size_t need = tri_part_bytes(dtype, n, batch);
    void* scr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scr_mu);
        if ((int)g_scr.size() <= dev) g_scr.resize(dev + 1, {nullptr, 0});
        auto& slot = g_scr[dev];
        if (slot.second < need) {
            ADI_HIP(hipStreamSynchronize(st));
            if (slot.first) (void)hipFree(slot.first);
            slot = {nullptr, 0};
            if (hipMalloc(&slot.first, need) != hipSuccess) {
                (void)hipGetLastError();
                slot.first = nullptr;
                return fail(ADI_ENOMEM, "hipMalloc of batched-solve scratch failed");
            }
            slot.second = need;
        }
        scr = slot.first;
    }
    return tri_run_part(dtype, n, batch, a, b, c, d, sys_stride, elem_stride, scr, st);
}

adi_status tridiag_solve_batched_noalloc(adi_dtype dtype, int n, int batch, const void* a, const void* b,
                                         const void* c, void* d, long long sys_stride,
                                         long long elem_stride, void* hip_stream)
{
    bool wg = false;
    TPlan p{};
    if (adi_status s = tri_check(dtype, n, batch, a, b, c, d, sys_stride, elem_stride, &wg, &p)) return s;
    if (n == 0 || batch == 0) return ADI_OK;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (wg) return tri_run_wg(dtype, p, n, batch, a, b, c, d, sys_stride, elem_stride, st);
    const size_t need = tri_part_bytes(dtype, n, batch);
    if (need > kNoAllocScratchBytes)
        return fail(ADI_EINVAL, "the layout needs " + std::to_string(need) +
                                    " bytes of partition workspace, above the no-allocation scratch of " +
                                    std::to_string(kNoAllocScratchBytes) + " bytes");
    void* scr = nullptr;
    if (adi_status s = noalloc_scratch(&scr)) return s;
    return tri_run_part(dtype, n, batch, a, b, c, d, sys_stride, elem_stride, scr, st);
}

}  // extern "C"

#include "batch.hpp"
#include "adjoint.hpp"
#include "tdc.hpp"
#include "split.hpp"
