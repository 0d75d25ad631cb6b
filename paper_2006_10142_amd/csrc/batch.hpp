// batch.hpp -- many independent simulations of uneven grid sizes advanced
// together: every launch of a step covers all simulations through a work list
// of (simulation, tile) items walked by a persistent grid.  Included at the end
// of adiwave.hip (same translation unit: it reuses the plain path's helpers).
//
// A batch step runs the same three kernels as the plain step (fused x-sweep,
// y-interface solve, y-chunk solve + update) on each simulation's own grid,
// coefficient and workspace; the per-simulation state lives in one device
// table of descriptors.  The two time levels of simulation s are lev[0] and
// lev[1]; at step parity p, lev[p] holds u^{n-1} (and receives u^{n+1}) and
// lev[p^1] holds u^n.  A hipGraph of two steps (both parities) can be captured
// and replayed.

namespace adw {

constexpr int kBatchStripRows = 1024;   // longest strip segment of a batched simulation

template <typename T>
struct SimDesc {
    int nx, ny, nseg, K, nxp, vec;
    int f_wt, f_tx, f_tiles;   // one-pass tiles (see fused.hpp)
    int f4_wt, f4_tx, f4_tiles;   // one-pass tiles with four nodes per lane (fused4.hpp)
    int s_wt, s_tx, s_hs, s_tiles;   // one-pass column strips (fusedr.hpp): width, strips, segment rows
    T* r;
    T* w;
    T* qin;
    T* sum;
    T* X;
    T* lev[2];
};

template <typename T>
struct BatchArgs {
    const SimDesc<T>* sims;
    const int2* items;    // work list of this launch: (simulation, tile)
    int nitems;
    int M, RS;            // chunk rows, fused strip rows
    int u_slot;           // level read as u^n
    int v_slot;           // level read as v (< 0: none)
    int out_slot;         // level written
    T alpha, beta, rho_scale;
};

// one-pass step of every simulation: work list of (simulation, tile), one tile
// per workgroup (FP32)
struct FBatchArgs {
    const SimDesc<float>* sims;
    const int2* items;
    int nitems;
    int u_slot, out_slot;   // level read as u^n; level holding u^{n-1}, receiving u^{n+1}
};

__global__ void __launch_bounds__(1024) k_fused_batch(FBatchArgs B)
{
    __shared__ FShared sh;
    const int it = xcd_band(blockIdx.x);
    if (it >= B.nitems) return;
    const int2 wi = B.items[it];
    const SimDesc<float>& S = B.sims[wi.x];
    FArgs A{};
    A.uc = S.lev[B.u_slot];
    A.up = S.lev[B.out_slot];
    A.r = S.r;
    A.qin = S.qin;
    A.nx = __builtin_amdgcn_readfirstlane(S.nx);
    A.ny = __builtin_amdgcn_readfirstlane(S.ny);
    A.nseg = __builtin_amdgcn_readfirstlane(S.nseg);
    A.wt = __builtin_amdgcn_readfirstlane(S.f_wt);
    A.tiles_x = __builtin_amdgcn_readfirstlane(S.f_tx);
    A.tiles = __builtin_amdgcn_readfirstlane(S.f_tiles);
    fused_tile(A, __builtin_amdgcn_readfirstlane(wi.y), sh);
}

// the same with four nodes per lane (each simulation's fused4.hpp tiles)
__global__ void __launch_bounds__(1024) k_fused4_batch(FBatchArgs B)
{
    __shared__ FShared4 sh;
    const int it = xcd_band(blockIdx.x);
    if (it >= B.nitems) return;
    const int2 wi = B.items[it];
    const SimDesc<float>& S = B.sims[wi.x];
    FArgs A{};
    A.uc = S.lev[B.u_slot];
    A.up = S.lev[B.out_slot];
    A.r = S.r;
    A.qin = S.qin;
    A.nx = __builtin_amdgcn_readfirstlane(S.nx);
    A.ny = __builtin_amdgcn_readfirstlane(S.ny);
    A.nseg = __builtin_amdgcn_readfirstlane(S.nseg);
    A.wt = __builtin_amdgcn_readfirstlane(S.f4_wt);
    A.tiles_x = __builtin_amdgcn_readfirstlane(S.f4_tx);
    A.tiles = __builtin_amdgcn_readfirstlane(S.f4_tiles);
    fused4_tile(A, __builtin_amdgcn_readfirstlane(wi.y), sh);
}

// the one-pass step on column strips (fusedr.hpp): work list of (simulation,
// strip segment), one per workgroup, in the order the host dealt it (block k
// takes item k: the XCD queues interleaved, padding items (-1, -1)); each
// simulation's strips are of one width (the last one cut by the grid's edge),
// so a plain handle tuned to the same width and segment rows runs the same
// arithmetic
__global__ void __launch_bounds__(Fr<float>::THREADS) k_fusedr_batch(FBatchArgs B)
{
    __shared__ FRShared<float> sh;
    const int it = blockIdx.x;
    if (it >= B.nitems) return;
    const int2 wi = B.items[it];
    if (wi.x < 0) return;
    const SimDesc<float>& S = B.sims[wi.x];
    FArgsT<float> A{};
    A.uc = S.lev[B.u_slot];
    A.up = S.lev[B.out_slot];
    A.r = S.r;
    A.qin = S.qin;
    A.nx = __builtin_amdgcn_readfirstlane(S.nx);
    A.ny = __builtin_amdgcn_readfirstlane(S.ny);
    A.nseg = __builtin_amdgcn_readfirstlane(S.nseg);
    A.wt = __builtin_amdgcn_readfirstlane(S.s_wt);
    A.tiles_x = __builtin_amdgcn_readfirstlane(S.s_tx);
    A.wide = A.tiles_x;
    A.hs = __builtin_amdgcn_readfirstlane(S.s_hs);
    A.tiles = __builtin_amdgcn_readfirstlane(S.s_tiles);
    fusedr_strip<float>(A, __builtin_amdgcn_readfirstlane(wi.y), sh);
}

template <typename T, int TR>
__global__ void __launch_bounds__(TR >= 256 ? TR : 256) k_xsweep_batch(BatchArgs<T> B)
{
    constexpr int G = (TR >= 256 ? TR : 256) / TR;
    __shared__ XShared<T, TR, true> sh[G];
    const int g = __builtin_amdgcn_readfirstlane(threadIdx.x / TR);
    const int t = threadIdx.x - g * TR;
    for (int base = blockIdx.x * G; base < B.nitems; base += gridDim.x * G) {
        const int it = base + g;
        XArgs<T> A{};
        int strip = 0;
        if (it < B.nitems) {
            const int2 wi = B.items[it];
            const SimDesc<T> S = B.sims[wi.x];
            A.u = S.lev[B.u_slot];
            A.r = S.r;
            A.qin = S.qin;
            A.w = S.w;
            A.nx = S.nx;
            A.ny = S.ny;
            A.nseg = S.nseg;
            A.vec = S.vec;
            A.sum = S.sum;
            A.K = S.K;
            A.nxp = S.nxp;
            strip = wi.y;
        } else {            // idle group: no rows, but the same barrier sequence
            A.nx = 1;
            A.ny = 0;
            A.nseg = 1;
        }
        A.rows_per_strip = B.RS;
        A.M = B.M;
        A.rho_scale = B.rho_scale;
        __syncthreads();    // the previous item's LDS use is over
        xsweep_strip<T, TR, true>(A, strip, t, sh[g]);
    }
}

template <typename T>
__device__ __forceinline__ YArgs<T> batch_yargs(const BatchArgs<T>& B, const SimDesc<T>& S)
{
    YArgs<T> a{};
    a.w = S.w;
    a.r = S.r;
    a.nx = S.nx;
    a.ny = S.ny;
    a.M = B.M;
    a.K = S.K;
    a.nxp = S.nxp;
    a.sum = S.sum;
    a.X = S.X;
    a.u = S.lev[B.u_slot];
    a.v = B.v_slot >= 0 ? S.lev[B.v_slot] : nullptr;
    a.out = S.lev[B.out_slot];
    a.alpha = B.alpha;
    a.beta = B.beta;
    return a;
}

template <typename T, int SK, int P>
__global__ void __launch_bounds__(kPB * P) k_yscan_batch(BatchArgs<T> B)
{
    __shared__ T lds[partition_lds_slots<P>() * kPB];
    for (int it = blockIdx.x; it < B.nitems; it += gridDim.x) {
        const int2 wi = B.items[it];
        const SimDesc<T> S = B.sims[wi.x];
        const YArgs<T> A = batch_yargs(B, S);
        __syncthreads();
        yscan_block<T, SK, P>(A, wi.y, lds);
    }
}

// items: (simulation, column block * K + chunk), 256 columns per block
template <typename T, int M, int GR>
__global__ void __launch_bounds__(256) k_ysolve_batch(BatchArgs<T> B)
{
    for (int it = blockIdx.x; it < B.nitems; it += gridDim.x) {
        const int2 wi = B.items[it];
        const SimDesc<T> S = B.sims[wi.x];
        const int cb = wi.y / S.K;
        const int c = wi.y - cb * S.K;
        const int i = cb * 256 + threadIdx.x;
        if (i < S.nx) ysolve_item<T, M, GR>(batch_yargs(B, S), i, c);
    }
}

}  // namespace adw

// ------------------------------------------------------------ host side ----
struct adi_batch_s {
    int count = 0;
    adi_dtype dtype = ADI_F32;
    hipStream_t stream = nullptr;
    std::vector<int> nx, ny;
    std::vector<double> h, dt;
    std::vector<adi_wave_s> sims;   // per-simulation views into the pools (not owners)
    void* pool = nullptr;           // every simulation's workspace
    void* desc = nullptr;           // device SimDesc table
    std::vector<unsigned char> desc_host;
    int2* items = nullptr;          // device work lists: x | yscan | ysolve
    int nx_items = 0, nys_items = 0, nyv_items = 0;
    int M = 32, RS = 32, max_nx = 0, max_K = 0;
    int x_tr = 256;
    YScanPlan yq{};
    int x_grid = 0, ys_grid = 0, yv_grid = 0;   // 0: one work unit per workgroup
    int parity = 0;
    long long steps_done = 0;       // steps since the last bind
    bool bound = false;
    std::vector<void*> lev0, lev1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    size_t bytes = 0;
    long long nodes = 0;
    // one-pass step: allowed when every simulation allows it (FP32, bound holds)
    int fused_ok = 0, fused = 0;
    int flane = 8;                  // nodes per lane of the one-pass tiles (8 or 4)
    int fstrips = 0;                // 1: the one-pass step on column strips instead of tiles
    int2* fitems = nullptr;         // (simulation, tile) of the eight-node tiles, then the four-node
                                    // ones, then (simulation, strip segment) of the column strips
    int nf_items = 0, nf4_items = 0, nfs_items = 0;   // list lengths (the strips' with padding)
    int nfs_segments = 0;           // strip segments over all simulations
    std::vector<int> s_wt, s_tx, s_hs, s_tiles;   // column-strip plan of every simulation
};

namespace {

void batch_free(adi_batch_s* b)
{
    if (b->fitems) (void)hipFree(b->fitems);
    b->fitems = nullptr;
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->pool) (void)hipFree(b->pool);
    if (b->desc) (void)hipFree(b->desc);
    if (b->items) (void)hipFree(b->items);
    b->gexec = nullptr; b->graph = nullptr;
    b->pool = b->desc = nullptr;
    b->items = nullptr;
}

bool batch_fits(int tr, adi_dtype dt) { return fuse_fits(tr, dt); }

// One-pass column strips of one simulation of a batch: the fewest strips of at
// most 240 columns, all of one width (a multiple of 8; the last strip is cut by
// the grid's edge), and segments of equal length, at most kBatchStripRows rows.
// The many simulations fill the device, so no segment count per compute unit is
// sought (the plain plan's rule).
void batch_strip_plan(int nx, int ny, int& wt, int& tx, int& hs, int& tiles)
{
    tx = (nx + kFrS - 1) / kFrS;
    wt = std::min(kFrS, ((nx + tx - 1) / tx + 7) / 8 * 8);
    tx = (nx + wt - 1) / wt;
    const int seg = (ny + kBatchStripRows - 1) / kBatchStripRows;
    hs = (ny + seg - 1) / seg;
    tiles = tx * ((ny + hs - 1) / hs);
}

template <typename T>
void fill_desc(adi_batch_s* b)
{
    b->desc_host.resize(sizeof(SimDesc<T>) * b->count);
    SimDesc<T>* d = reinterpret_cast<SimDesc<T>*>(b->desc_host.data());
    for (int s = 0; s < b->count; ++s) {
        const adi_wave_s& w = b->sims[s];
        d[s].nx = w.nx; d[s].ny = w.ny; d[s].nseg = w.nseg; d[s].K = w.K; d[s].nxp = w.nxp;
        d[s].f_wt = w.f_wt; d[s].f_tx = w.f_tx; d[s].f_tiles = w.f_tiles;
        d[s].f4_wt = w.f4_wt; d[s].f4_tx = w.f4_tx; d[s].f4_tiles = w.f4_tiles;
        if (!b->s_wt.empty()) {
            d[s].s_wt = b->s_wt[s]; d[s].s_tx = b->s_tx[s]; d[s].s_hs = b->s_hs[s]; d[s].s_tiles = b->s_tiles[s];
        }
        d[s].vec = ((size_t)w.nx * sizeof(T)) % 16 == 0;
        d[s].r = (T*)w.r; d[s].w = (T*)w.w; d[s].qin = (T*)w.qin; d[s].sum = (T*)w.sum; d[s].X = (T*)w.X;
        d[s].lev[0] = b->bound ? (T*)b->lev0[s] : nullptr;
        d[s].lev[1] = b->bound ? (T*)b->lev1[s] : nullptr;
        if (b->bound)
            d[s].vec = d[s].vec && aligned16(b->lev0[s]) && aligned16(b->lev1[s]) && aligned16(w.r) &&
                       aligned16(w.w);
    }
}

adi_status batch_upload(adi_batch_s* b)
{
    if (b->dtype == ADI_F32) fill_desc<float>(b);
    else fill_desc<double>(b);
    ADI_HIP(hipMemcpyAsync(b->desc, b->desc_host.data(), b->desc_host.size(), hipMemcpyHostToDevice,
                           b->stream));
    ADI_HIP(hipStreamSynchronize(b->stream));
    return ADI_OK;
}

int units(int nitems, int per) { return (nitems + per - 1) / per; }

template <typename T, int TR>
void launch_xb1(int grid, const BatchArgs<T>& a, hipStream_t st)
{
    constexpr int NT = TR >= 256 ? TR : 256;
    hipLaunchKernelGGL((k_xsweep_batch<T, TR>), dim3(grid), dim3(NT), 0, st, a);
}

template <typename T>
adi_status queue_batch_solve(adi_batch_s* b, int u_slot, int v_slot, int out_slot, T alpha, T beta,
                             T rho, hipStream_t st)
{
    BatchArgs<T> a{};
    a.sims = static_cast<const SimDesc<T>*>(b->desc);
    a.M = b->M;
    a.RS = b->RS;
    a.u_slot = u_slot; a.v_slot = v_slot; a.out_slot = out_slot;
    a.alpha = alpha; a.beta = beta; a.rho_scale = rho;

    a.items = b->items;
    a.nitems = b->nx_items;
    const int G = x_groups_per_wg(b->x_tr);
    const int xu = units(b->nx_items, G);
    const int xg = b->x_grid > 0 ? std::min(b->x_grid, xu) : xu;
    switch (b->x_tr) {
        case 64: launch_xb1<T, 64>(xg, a, st); break;
        case 128: launch_xb1<T, 128>(xg, a, st); break;
        case 256: launch_xb1<T, 256>(xg, a, st); break;
        case 1024:
            if constexpr (sizeof(T) == 4) { launch_xb1<T, 1024>(xg, a, st); break; }
            return fail(ADI_EUNSUPPORTED, "no batched x-sweep for this plan");
        default: return fail(ADI_EUNSUPPORTED, "no batched x-sweep for this plan");
    }
    ADI_LAUNCHED("x_sweep_batch");

    a.items = b->items + b->nx_items;
    a.nitems = b->nys_items;
    const int sg = b->ys_grid > 0 ? std::min(b->ys_grid, b->nys_items) : b->nys_items;
    const dim3 sblk(kPB * b->yq.p);
    bool ok = true;
    if (b->yq.p == 16) {
        switch (b->yq.sk) {
            case 2: hipLaunchKernelGGL((k_yscan_batch<T, 2, 16>), dim3(sg), sblk, 0, st, a); break;
            case 4: hipLaunchKernelGGL((k_yscan_batch<T, 4, 16>), dim3(sg), sblk, 0, st, a); break;
            case 8: hipLaunchKernelGGL((k_yscan_batch<T, 8, 16>), dim3(sg), sblk, 0, st, a); break;
            default: ok = false;
        }
    } else if (b->yq.p == 64) {
        switch (b->yq.sk) {
            case 4: hipLaunchKernelGGL((k_yscan_batch<T, 4, 64>), dim3(sg), sblk, 0, st, a); break;
            case 8: hipLaunchKernelGGL((k_yscan_batch<T, 8, 64>), dim3(sg), sblk, 0, st, a); break;
            default: ok = false;
        }
    } else ok = false;
    if (!ok) return fail(ADI_EUNSUPPORTED, "no batched y-interface kernel for this plan");
    ADI_LAUNCHED("y_scan_batch");

    a.items = b->items + b->nx_items + b->nys_items;
    a.nitems = b->nyv_items;
    const int vg = b->yv_grid > 0 ? std::min(b->yv_grid, b->nyv_items) : b->nyv_items;
    hipLaunchKernelGGL((k_ysolve_batch<T, 32, 8>), dim3(vg), dim3(256), 0, st, a);
    ADI_LAUNCHED("y_solve_batch");
    return ADI_OK;
}

adi_status batch_step_once(adi_batch_s* b, hipStream_t st, int parity)
{
    const int p = parity;
    if (b->fused && b->fstrips) {
        FBatchArgs a{static_cast<const SimDesc<float>*>(b->desc), b->fitems + b->nf_items + b->nf4_items,
                     b->nfs_items, p ^ 1, p};
        hipLaunchKernelGGL(k_fusedr_batch, dim3((b->nfs_items + 7) / 8 * 8), dim3(Fr<float>::THREADS), 0, st, a);
        ADI_LAUNCHED("fused_batch");
        return ADI_OK;
    }
    if (b->fused && b->flane == 4) {
        FBatchArgs a{static_cast<const SimDesc<float>*>(b->desc), b->fitems + b->nf_items, b->nf4_items, p ^ 1, p};
        hipLaunchKernelGGL(k_fused4_batch, dim3((b->nf4_items + 7) / 8 * 8), dim3(1024), 0, st, a);
        ADI_LAUNCHED("fused_batch");
        return ADI_OK;
    }
    if (b->fused) {
        FBatchArgs a{static_cast<const SimDesc<float>*>(b->desc), b->fitems, b->nf_items, p ^ 1, p};
        hipLaunchKernelGGL(k_fused_batch, dim3((b->nf_items + 7) / 8 * 8), dim3(1024), 0, st, a);
        ADI_LAUNCHED("fused_batch");
        return ADI_OK;
    }
    return b->dtype == ADI_F32
               ? queue_batch_solve<float>(b, p ^ 1, p, p, 2.f, -1.f, 1.f, st)
               : queue_batch_solve<double>(b, p ^ 1, p, p, 2.0, -1.0, 1.0, st);
}

void batch_drop_graph(adi_batch_s* b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
}

adi_status batch_capture(adi_batch_s* b)
{
    batch_drop_graph(b);
    hipStream_t cs = nullptr;
    ADI_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    adi_status s = ADI_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return fail(ADI_EHIP, "hipStreamBeginCapture failed");
    }
    s = batch_step_once(b, cs, 0);
    if (s == ADI_OK) s = batch_step_once(b, cs, 1);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (s != ADI_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess || !g) return fail(ADI_EHIP, "hipStreamEndCapture failed");
    if (hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        b->gexec = nullptr;
        return fail(ADI_EHIP, "hipGraphInstantiate failed");
    }
    b->graph = g;
    return ADI_OK;
}

// per-simulation creation work (coefficient, pivots, static planes)
template <typename T>
adi_status batch_setup_sim(adi_wave_s* w, const void* speed, double scalar)
{
    return set_coef<T>(w, speed, scalar, 1);
}

}  // namespace

extern "C" {

adi_status adi_batch_create(adi_batch_t* out, int count, const int* nx, const int* ny, const double* h,
                            const double* dt, const void* const* speed, const double* speed_scalar,
                            adi_dtype dtype, void* hip_stream)
{
    if (!out) return fail(ADI_EINVAL, "out is null");
    *out = nullptr;
    if (count < 1) return fail(ADI_EINVAL, "count must be >= 1");
    if (!nx || !ny || !h || !dt) return fail(ADI_EINVAL, "null size array");
    if (dtype != ADI_F32 && dtype != ADI_F64) return fail(ADI_EINVAL, "unknown dtype");
    int max_nx = 0;
    for (int s = 0; s < count; ++s) {
        if (nx[s] < 1 || ny[s] < 1) return fail(ADI_EINVAL, "every nx, ny must be >= 1");
        if (nx[s] > 8192 || ny[s] > 16384) return fail(ADI_EUNSUPPORTED, "grid larger than 8192 x 16384");
        if (!finite_pos(h[s]) || !finite_pos(dt[s])) return fail(ADI_EINVAL, "h and dt must be finite and > 0");
        const bool has_field = speed && speed[s];
        if (!has_field && !(speed_scalar && finite_pos(speed_scalar[s])))
            return fail(ADI_EINVAL, "a simulation has neither a speed field nor a positive scalar speed");
        max_nx = std::max(max_nx, nx[s]);
    }
    XPlan xp{};
    if (!choose_x(max_nx, dtype, xp)) return fail(ADI_EUNSUPPORTED, "nx > 8192");
    if (!batch_fits(xp.tr, dtype))
        return fail(ADI_EUNSUPPORTED, "the widest grid does not fit the batched x-sweep in LDS");

    adi_batch_s* b = new adi_batch_s();
    b->count = count;
    b->dtype = dtype;
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->nx.assign(nx, nx + count);
    b->ny.assign(ny, ny + count);
    b->h.assign(h, h + count);
    b->dt.assign(dt, dt + count);
    b->x_tr = xp.tr;
    b->max_nx = max_nx;
    b->sims.resize(count);
    const size_t es = esize(dtype);
    // carve every simulation's workspace out of one pool (256-byte aligned parts)
    auto al = [](size_t n) { return (n + 63) & ~size_t(63); };   // elements, 256 B for f32
    std::vector<size_t> off(count);
    size_t total = 0;
    for (int s = 0; s < count; ++s) {
        adi_wave_s& w = b->sims[s];
        w.nx = nx[s]; w.ny = ny[s]; w.h = h[s]; w.dt = dt[s]; w.dtype = dtype;
        w.stream = b->stream;
        w.M = b->M;
        w.K = (ny[s] + w.M - 1) / w.M;
        w.nxp = (nx[s] + kPB - 1) / kPB * kPB;
        w.nseg = (nx[s] + kSeg - 1) / kSeg;
        w.xp = xp;
        w.xp.fuse = 1;
        w.xp.frs = b->RS;
        w.w_cap = std::max((size_t)nx[s] * ny[s], (size_t)5 * w.K * nx[s]);
        b->max_K = std::max(b->max_K, w.K);
        off[s] = total;
        total += al((size_t)nx[s] * ny[s]) + al(w.w_cap) + al((size_t)ny[s] * w.nseg) +
                 al((size_t)kSummaryPlanes * w.K * w.nxp) + al((size_t)w.K * nx[s]);
        b->nodes += (long long)nx[s] * ny[s];
    }
    if (!choose_yscan(b->max_K, b->yq)) {
        delete b;
        return fail(ADI_EUNSUPPORTED, "too many y-chunks for the interface solver");
    }
    if (hipMalloc(&b->pool, total * es) != hipSuccess ||
        hipMalloc(&b->desc, (dtype == ADI_F32 ? sizeof(SimDesc<float>) : sizeof(SimDesc<double>)) * count) !=
            hipSuccess) {
        (void)hipGetLastError();
        batch_free(b);
        delete b;
        return fail(ADI_ENOMEM, "hipMalloc of the batch workspace failed");
    }
    b->bytes = total * es;
    for (int s = 0; s < count; ++s) {
        adi_wave_s& w = b->sims[s];
        char* p = static_cast<char*>(b->pool) + off[s] * es;
        auto take = [&](size_t n) { void* q = p; p += al(n) * es; return q; };
        w.r = take((size_t)nx[s] * ny[s]);
        w.w = take(w.w_cap);
        w.qin = take((size_t)ny[s] * w.nseg);
        w.sum = take((size_t)kSummaryPlanes * w.K * w.nxp);
        w.X = take((size_t)w.K * nx[s]);
        w.yq = b->yq;
    }
    // work lists, in simulation order
    std::vector<int2> items;
    for (int s = 0; s < count; ++s)
        for (int st = 0; st < (ny[s] + b->RS - 1) / b->RS; ++st) items.push_back(make_int2(s, st));
    b->nx_items = (int)items.size();
    for (int s = 0; s < count; ++s)
        for (int blk = 0; blk < b->sims[s].nxp / kPB; ++blk) items.push_back(make_int2(s, blk));
    b->nys_items = (int)items.size() - b->nx_items;
    for (int s = 0; s < count; ++s)
        for (int cb = 0; cb < (nx[s] + 255) / 256; ++cb)
            for (int c = 0; c < b->sims[s].K; ++c) items.push_back(make_int2(s, cb * b->sims[s].K + c));
    b->nyv_items = (int)items.size() - b->nx_items - b->nys_items;
    adi_status st = ADI_OK;
    if (hipMalloc(&b->items, items.size() * sizeof(int2)) != hipSuccess) {
        (void)hipGetLastError();
        st = fail(ADI_ENOMEM, "hipMalloc of the work lists failed");
    }
    if (st == ADI_OK &&
        hipMemcpyAsync(b->items, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream) !=
            hipSuccess)
        st = fail(ADI_EHIP, "upload of the work lists failed");
    for (int s = 0; s < count && st == ADI_OK; ++s) {
        const void* f = speed ? speed[s] : nullptr;
        const double sc = speed_scalar ? speed_scalar[s] : 1.0;
        st = dtype == ADI_F32 ? batch_setup_sim<float>(&b->sims[s], f, sc)
                              : batch_setup_sim<double>(&b->sims[s], f, sc);
    }
    if (st == ADI_OK) {
        // one-pass tiles of every simulation (each view's plan was set with its r)
        b->fused_ok = dtype == ADI_F32 ? 1 : 0;
        std::vector<int2> fi;
        for (int s = 0; s < count && b->fused_ok; ++s) {
            if (!b->sims[s].fused_ok) b->fused_ok = 0;
            for (int tl = 0; tl < b->sims[s].f_tiles; ++tl) fi.push_back(make_int2(s, tl));
        }
        b->nf_items = (int)fi.size();
        for (int s = 0; s < count && b->fused_ok; ++s)
            for (int tl = 0; tl < b->sims[s].f4_tiles; ++tl) fi.push_back(make_int2(s, tl));
        b->nf4_items = (int)fi.size() - b->nf_items;
        b->s_wt.assign(count, 0); b->s_tx.assign(count, 0); b->s_hs.assign(count, 0); b->s_tiles.assign(count, 0);
        for (int s = 0; s < count && b->fused_ok; ++s) {
            batch_strip_plan(nx[s], ny[s], b->s_wt[s], b->s_tx[s], b->s_hs[s], b->s_tiles[s]);
            for (int tl = 0; tl < b->s_tiles[s]; ++tl) fi.push_back(make_int2(s, tl));
        }
        b->nfs_items = (int)fi.size() - b->nf_items - b->nf4_items;
        {
            // Load balance: whole simulations are dealt to 8 queues, one per XCD, the
            // largest first to the least loaded queue (so a simulation's neighbouring
            // strips share one L2), and each queue runs its longest segments first, so
            // that the short ones fill in at the end.  Block k of the launch takes
            // entry k / 8 of queue k mod 8 (the hardware hands blocks to the XCDs in
            // turn); entries past a queue's end are (-1, -1).  Cost of a segment: its
            // x-window columns times its x-rows.
            auto cost = [&](int2 q) {
                const int s = q.x, r0 = (q.y / b->s_tx[s]) * b->s_hs[s];
                return (long long)(b->s_wt[s] + 2 * kFuKx) * (std::min(b->s_hs[s], ny[s] - r0) + 2 * kFuKy);
            };
            b->nfs_segments = b->nfs_items;
            std::vector<int2> strip(fi.end() - b->nfs_items, fi.end());
            fi.resize(fi.size() - b->nfs_items);
            std::vector<long long> scost(count, 0);
            std::vector<std::vector<int2>> per(count);
            for (const int2& q : strip) {
                scost[q.x] += cost(q);
                per[q.x].push_back(q);
            }
            std::vector<int> ord;
            for (int s = 0; s < count; ++s)
                if (scost[s] > 0) ord.push_back(s);
            std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return scost[x] > scost[y]; });
            std::vector<std::vector<int2>> qs(8);
            std::vector<long long> load(8, 0);
            for (int s : ord) {
                const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                for (const int2& q : per[s]) qs[x].push_back(q);
                load[x] += scost[s];
            }
            size_t len = 0;
            for (auto& q : qs) {
                std::stable_sort(q.begin(), q.end(), [&](int2 x, int2 y) { return cost(x) > cost(y); });
                len = std::max(len, q.size());
            }
            for (size_t k = 0; k < len; ++k)
                for (int x = 0; x < 8; ++x) fi.push_back(k < qs[x].size() ? qs[x][k] : make_int2(-1, -1));
            b->nfs_items = (int)(8 * len);
        }
        if (b->fused_ok) {
            if (hipMalloc(&b->fitems, fi.size() * sizeof(int2)) != hipSuccess) {
                (void)hipGetLastError();
                b->fitems = nullptr;
                st = fail(ADI_ENOMEM, "hipMalloc of the one-pass work list failed");
            } else if (hipMemcpyAsync(b->fitems, fi.data(), fi.size() * sizeof(int2), hipMemcpyHostToDevice,
                                      b->stream) != hipSuccess) {
                st = fail(ADI_EHIP, "upload of the one-pass work list failed");
            }
            b->fused = st == ADI_OK ? 1 : 0;
        }
    }
    if (st == ADI_OK) st = batch_upload(b);
    if (st != ADI_OK) {
        batch_free(b);
        delete b;
        return st;
    }
    *out = b;
    return ADI_OK;
}

adi_status adi_batch_bind(adi_batch_t b, void* const* u_prev, void* const* u_curr)
{
    if (!b) return fail(ADI_EINVAL, "null batch");
    if (!u_prev || !u_curr) return fail(ADI_EINVAL, "null level arrays");
    for (int s = 0; s < b->count; ++s)
        if (!u_prev[s] || !u_curr[s] || u_prev[s] == u_curr[s])
            return fail(ADI_EINVAL, "every simulation needs two distinct non-null levels");
    b->lev0.assign(u_prev, u_prev + b->count);
    b->lev1.assign(u_curr, u_curr + b->count);
    b->bound = true;
    b->parity = 0;
    b->steps_done = 0;
    batch_drop_graph(b);
    return batch_upload(b);
}

adi_status adi_batch_start(adi_batch_t b, int mode)
{
    if (!b) return fail(ADI_EINVAL, "null batch");
    if (!b->bound) return fail(ADI_EINVAL, "bind the levels first");
    if (mode != ADI_START_PAPER && mode != ADI_START_GHOST) return fail(ADI_EINVAL, "unknown start mode");
    if (b->steps_done != 0) return fail(ADI_EINVAL, "start must precede the steps (rebind to restart)");
    if (mode == ADI_START_PAPER) {
        for (int s = 0; s < b->count; ++s)
            ADI_HIP(hipMemcpyAsync(b->lev1[s], b->lev0[s], (size_t)b->nx[s] * b->ny[s] * esize(b->dtype),
                                   hipMemcpyDeviceToDevice, b->stream));
        return ADI_OK;
    }
    return b->dtype == ADI_F32 ? queue_batch_solve<float>(b, 0, -1, 1, 1.f, 0.f, 0.5f, b->stream)
                               : queue_batch_solve<double>(b, 0, -1, 1, 1.0, 0.0, 0.5, b->stream);
}

adi_status adi_batch_step(adi_batch_t b, int nsteps)
{
    if (!b) return fail(ADI_EINVAL, "null batch");
    if (!b->bound) return fail(ADI_EINVAL, "bind the levels first");
    if (nsteps < 0) return fail(ADI_EINVAL, "nsteps must be >= 0");
    int left = nsteps;
    b->steps_done += nsteps;
    if (b->gexec && b->parity == 1 && left > 0) {
        if (adi_status s = batch_step_once(b, b->stream, 1)) return s;
        b->parity = 0;
        --left;
    }
    if (b->gexec) {
        for (; left >= 2; left -= 2) ADI_HIP(hipGraphLaunch(b->gexec, b->stream));
    }
    for (; left > 0; --left) {
        if (adi_status s = batch_step_once(b, b->stream, b->parity)) return s;
        b->parity ^= 1;
    }
    return ADI_OK;
}

adi_status adi_batch_levels(adi_batch_t b, void** u_prev, void** u_curr)
{
    if (!b) return fail(ADI_EINVAL, "null batch");
    if (!b->bound) return fail(ADI_EINVAL, "bind the levels first");
    if (!u_prev || !u_curr) return fail(ADI_EINVAL, "null output arrays");
    for (int s = 0; s < b->count; ++s) {
        u_prev[s] = b->parity == 0 ? b->lev0[s] : b->lev1[s];
        u_curr[s] = b->parity == 0 ? b->lev1[s] : b->lev0[s];
    }
    return ADI_OK;
}

adi_status adi_batch_graph(adi_batch_t b, int enable)
{
    if (!b) return fail(ADI_EINVAL, "null batch");
    if (!enable) {
        batch_drop_graph(b);
        return ADI_OK;
    }
    if (!b->bound) return fail(ADI_EINVAL, "bind the levels first");
    return batch_capture(b);
}

adi_status adi_batch_get_plan(adi_batch_t b, adi_batch_plan* p)
{
    if (!b || !p) return fail(ADI_EINVAL, "null argument");
    p->x_threads_per_line = b->x_tr;
    p->x_grid = b->x_grid;
    p->yscan_grid = b->ys_grid;
    p->ysolve_grid = b->yv_grid;
    p->graph = b->gexec != nullptr;
    p->count = b->count;
    p->nodes = b->nodes;
    p->workspace_bytes = b->bytes;
    p->x_items = b->nx_items;
    p->yscan_items = b->nys_items;
    p->ysolve_items = b->nyv_items;
    p->fused_step = b->fused;
    p->fused_allowed = b->fused_ok;
    p->fused_items = b->fstrips ? b->nfs_segments : b->flane == 4 ? b->nf4_items : b->nf_items;
    p->fused_lane_nodes = b->flane;
    p->fused_strips = b->fstrips;
    return ADI_OK;
}

adi_status adi_batch_set_plan(adi_batch_t b, const adi_batch_plan* p)
{
    if (!b || !p) return fail(ADI_EINVAL, "null argument");
    int tr = p->x_threads_per_line > 0 ? p->x_threads_per_line : b->x_tr;
    if (tr != 64 && tr != 128 && tr != 256 && tr != 1024)
        return fail(ADI_EINVAL, "x_threads_per_line must be 64, 128, 256 or 1024");
    if (8LL * tr < b->max_nx) return fail(ADI_EINVAL, "8 * x_threads_per_line must cover the widest grid");
    if (!batch_fits(tr, b->dtype)) return fail(ADI_EUNSUPPORTED, "plan does not fit in LDS");
    if (p->x_grid < 0 || p->yscan_grid < 0 || p->ysolve_grid < 0)
        return fail(ADI_EINVAL, "grid sizes must be >= 0");
    if (p->fused_step < 0 || p->fused_step > 2) return fail(ADI_EINVAL, "fused_step must be 0, 1 or 2");
    if (p->fused_step == 1 && !b->fused_ok)
        return fail(ADI_EUNSUPPORTED, "the one-pass step is not allowed for every simulation of the batch");
    if (p->fused_lane_nodes != 0 && p->fused_lane_nodes != 4 && p->fused_lane_nodes != 8)
        return fail(ADI_EINVAL, "fused_lane_nodes must be 0, 4 or 8");
    if (p->fused_strips < 0 || p->fused_strips > 2) return fail(ADI_EINVAL, "fused_strips must be 0, 1 or 2");
    if (p->fused_step > 0) b->fused = p->fused_step == 1 ? 1 : 0;
    if (p->fused_strips) b->fstrips = p->fused_strips == 1 ? 1 : 0;
    if (p->fused_lane_nodes) b->flane = p->fused_lane_nodes;
    b->x_tr = tr;
    b->x_grid = p->x_grid;
    b->ys_grid = p->yscan_grid;
    b->yv_grid = p->ysolve_grid;
    if (b->gexec) return batch_capture(b);   // keep the captured graph in step with the plan
    return ADI_OK;
}

adi_status adi_batch_autotune(adi_batch_t b, int trial_steps, double* best_ms)
{
    if (!b) return fail(ADI_EINVAL, "null batch");
    if (trial_steps < 2 || trial_steps > 1000) return fail(ADI_EINVAL, "trial_steps must be in [2, 1000]");
    // scratch levels so that the bound simulations are left untouched
    const size_t es = esize(b->dtype);
    size_t tot = 0;
    for (int s = 0; s < b->count; ++s) tot += ((size_t)b->nx[s] * b->ny[s] + 63) & ~size_t(63);
    void* scr = nullptr;
    if (hipMalloc(&scr, 2 * tot * es) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ADI_ENOMEM, "hipMalloc of autotuning scratch failed");
    }
    ADI_HIP(hipMemsetAsync(scr, 0, 2 * tot * es, b->stream));
    const bool was_bound = b->bound;
    std::vector<void*> keep0 = b->lev0, keep1 = b->lev1;
    const int keep_parity = b->parity;
    const bool had_graph = b->gexec != nullptr;
    batch_drop_graph(b);
    std::vector<void*> s0(b->count), s1(b->count);
    size_t o = 0;
    for (int s = 0; s < b->count; ++s) {
        s0[s] = static_cast<char*>(scr) + o * es;
        s1[s] = static_cast<char*>(scr) + (tot + o) * es;
        o += ((size_t)b->nx[s] * b->ny[s] + 63) & ~size_t(63);
    }
    b->lev0 = s0; b->lev1 = s1; b->bound = true; b->parity = 0;
    adi_status st = batch_upload(b);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (st == ADI_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        st = fail(ADI_EHIP, "hipEventCreate failed");
    auto trial = [&](double& ms) -> adi_status {
        if (adi_status s = batch_step_once(b, b->stream, 0)) return s;   // warm
        ADI_HIP(hipEventRecord(e0, b->stream));
        for (int k = 0; k < trial_steps; ++k)
            if (adi_status s = batch_step_once(b, b->stream, k & 1)) return s;
        ADI_HIP(hipEventRecord(e1, b->stream));
        ADI_HIP(hipEventSynchronize(e1));
        float f = 0.f;
        ADI_HIP(hipEventElapsedTime(&f, e0, e1));
        ms = f / trial_steps;
        return ADI_OK;
    };
    // candidates: line-group width, then each kernel's persistent grid in turn
    // (the one-pass step has no plan to choose: it is only timed)
    double best = 1e30;
    int btr = b->x_tr, bxg = b->x_grid, bsg = b->ys_grid, bvg = b->yv_grid;
    static const int grids[] = {0, 256, 512, 1024, 2048, 4096};
    if (st == ADI_OK && b->fused) {
        // the one-pass step: the fastest of its two tile kinds and the column strips
        int blane = b->flane, bstrips = b->fstrips;
        for (int kind : {8, 4, 0}) {
            b->fstrips = kind == 0 ? 1 : 0;
            if (kind) b->flane = kind;
            double ms = 0;
            if ((st = trial(ms)) != ADI_OK) break;
            if (ms < best) { best = ms; blane = b->flane; bstrips = b->fstrips; }
        }
        b->flane = blane;
        b->fstrips = bstrips;
    } else if (st == ADI_OK) {
        for (int tr : {128, 256, 1024}) {
            if (8LL * tr < b->max_nx || !batch_fits(tr, b->dtype)) continue;
            b->x_tr = tr; b->x_grid = 0; b->ys_grid = 0; b->yv_grid = 0;
            double ms = 0;
            if ((st = trial(ms)) != ADI_OK) break;
            if (ms < best) { best = ms; btr = tr; }
        }
        b->x_tr = btr;
        int* knobs[3] = {&b->x_grid, &b->ys_grid, &b->yv_grid};
        int* bests[3] = {&bxg, &bsg, &bvg};
        for (int q = 0; q < 3 && st == ADI_OK; ++q) {
            *bests[q] = 0;
            for (int gsz : grids) {
                *knobs[q] = gsz;
                double ms = 0;
                if ((st = trial(ms)) != ADI_OK) break;
                if (ms < best) { best = ms; *bests[q] = gsz; }
            }
            *knobs[q] = *bests[q];
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(b->stream);
    (void)hipFree(scr);
    b->x_tr = btr; b->x_grid = bxg; b->ys_grid = bsg; b->yv_grid = bvg;
    b->lev0 = keep0; b->lev1 = keep1; b->bound = was_bound; b->parity = keep_parity;
    if (adi_status s2 = batch_upload(b)) return st != ADI_OK ? st : s2;
    if (st == ADI_OK && had_graph && b->bound) st = batch_capture(b);
    if (st == ADI_OK && best_ms) *best_ms = best;
    return st;
}

adi_status adi_batch_destroy(adi_batch_t b)
{
    if (!b) return ADI_OK;
    (void)hipStreamSynchronize(b->stream);
    batch_free(b);
    delete b;
    return ADI_OK;
}

}  // extern "C"
