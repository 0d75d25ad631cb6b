// split.hpp -- paper-fidelity modes: the ADI split exactly as printed (eqs.
// (fr1)-(fr2)) and the line systems of Listing 1.  Levels sit on half steps: the
// x-sub-step takes (u^{k-1/2}, u^k) to u^{k+1/2} and the y-sub-step (u^k,
// u^{k+1/2}) to u^{k+1}; each is a three-level scheme with the tau^2 denominator
// and one direction's second difference D,
//     (u_new - 2 u_mid + u_old) / tau^2 - th_new kappa D u_new - th_old kappa D u_old = f,
// i.e. with r = tau^2 kappa / (2 h^2) the line system
//     -cn r u_new[k-1] + (1 + 2 cn r) u_new[k] - cn r u_new[k+1]
//         = 2 u_mid - u_old + co r (u_old[k-1] - 2 u_old[k] + u_old[k+1]) + tau^2 f,
// cn = 2 th_new, co = 2 th_old.  Eqs. (fr1)-(fr2) weigh the new and the oldest
// level by 1/2 (cn = co = 1); Listing 1 (a = c = tau^2, b = 2 tau^2 + h^2, a
// right-hand side from the older levels only) is th_new = 1, th_old = 0 (cn = 2,
// co = 0).  The lines are solved by the cyclic-reduction kernels of cr.hpp, the
// paper's own solver.  Included at the end of adiwave.hip.

namespace adw {

// coefficients and right-hand side of the x- (dir 0) or y-lines (dir 1) of one
// sub-step, without the couplings past the grid edge
template <typename T>
__global__ void __launch_bounds__(256) k_split_setup(const T* __restrict__ u_old, const T* __restrict__ u_mid,
                                                     const T* __restrict__ r, T* a, T* b, T* c, T* d, int nx,
                                                     int ny, int dir, T cn, T co)
{
    const long long n = (long long)nx * ny;
    const long long st = dir == 0 ? 1 : nx;
    for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < n; p += (long long)gridDim.x * 256) {
        const int j = (int)(p / nx), i = (int)(p - (long long)j * nx);
        const bool first = dir == 0 ? i == 0 : j == 0;
        const bool last = dir == 0 ? i == nx - 1 : j == ny - 1;
        const T rr = r[p];
        const T g = cn * rr;
        a[p] = first ? T(0) : -g;
        c[p] = last ? T(0) : -g;
        b[p] = T(1) + T(2) * g;
        const T uo = u_old[p];
        const T lo = first ? T(0) : u_old[p - st], hi = last ? T(0) : u_old[p + st];
        d[p] = fma_rn(co * rr, (lo + hi) - T(2) * uo, T(2) * u_mid[p] - uo);
    }
}

}  // namespace adw

namespace {

template <typename T>
adi_status split_substep(adi_wave_s* w, int dir, const void* u_old, const void* u_mid, void* u_new, T cn, T co,
                         const adi_source* f)
{
    const long long n = (long long)w->nx * w->ny;
    T* a = static_cast<T*>(w->cr_abc);
    T* b = a + n;
    T* c = b + n;
    T* d = static_cast<T*>(w->w);
    hipLaunchKernelGGL((k_split_setup<T>), dim3(cr_grid(n)), dim3(256), 0, w->stream, static_cast<const T*>(u_old),
                       static_cast<const T*>(u_mid), static_cast<const T*>(w->r), a, b, c, d, w->nx, w->ny, dir, cn,
                       co);
    ADI_LAUNCHED(dir == 0 ? "split_setup_x" : "split_setup_y");
    if (f && f->count > 0) {
        hipLaunchKernelGGL((k_cr_sources<T>), dim3(1), dim3(64), 0, w->stream, d, f->idx,
                           static_cast<const T*>(f->amp), f->count, (T)(w->dt * w->dt), n);
        ADI_LAUNCHED("split_sources");
    }
    CrArgs<T> L = dir == 0 ? CrArgs<T>{a, b, c, d, w->nx, w->ny, (long long)w->nx, 1LL, 0}
                           : CrArgs<T>{a, b, c, d, w->ny, w->nx, 1LL, (long long)w->nx, 0};
    if (adi_status s = queue_cr_lines<T>(w, L)) return s;
    ADI_HIP(hipMemcpyAsync(u_new, d, (size_t)n * sizeof(T), hipMemcpyDeviceToDevice, w->stream));
    return ADI_OK;
}

template <typename T>
adi_status do_step_split(adi_wave_s* w, int mode, void* u_half, void* u_curr, const adi_source* f,
                         const adi_source* f_half, const adi_receivers* rec)
{
    if (!w->cr_abc) {
        const size_t bytes = 3 * (size_t)w->nx * w->ny * sizeof(T);
        if (hipMalloc(&w->cr_abc, bytes) != hipSuccess) {
            (void)hipGetLastError();
            w->cr_abc = nullptr;
            return fail(ADI_ENOMEM, "hipMalloc of the line coefficients failed");
        }
        w->bytes += bytes;
    }
    const T cn = mode == ADI_SPLIT_FR ? T(1) : T(2);
    const T co = mode == ADI_SPLIT_FR ? T(1) : T(0);
    // x-sub-step: (u^{k-1/2}, u^k) -> u^{k+1/2}, written over u^{k-1/2}
    if (adi_status s = split_substep<T>(w, 0, u_half, u_curr, u_half, cn, co, f)) return s;
    // y-sub-step: (u^k, u^{k+1/2}) -> u^{k+1}, written over u^k
    if (adi_status s = split_substep<T>(w, 1, u_curr, u_half, u_curr, cn, co, f_half)) return s;
    if (rec && rec->count > 0) {
        hipLaunchKernelGGL((k_record<T>), dim3((rec->count + 255) / 256), dim3(256), 0, w->stream,
                           static_cast<const T*>(u_curr), rec->idx, static_cast<T*>(rec->traces), rec->count,
                           (long long)w->nx * w->ny);
        ADI_LAUNCHED("record");
    }
    return ADI_OK;
}

}  // namespace

extern "C" {

adi_status adi_wave_step_split(adi_wave_t w, int mode, void* u_half, void* u_curr, const adi_source* f,
                               const adi_source* f_half, const adi_receivers* rec)
{
    if (adi_status s = check_handle(w)) return s;
    if (mode != ADI_SPLIT_FR && mode != ADI_SPLIT_THETA1)
        return fail(ADI_EINVAL, "mode must be ADI_SPLIT_FR or ADI_SPLIT_THETA1");
    if (!u_half || !u_curr) return fail(ADI_EINVAL, "null level pointer");
    if (u_half == u_curr) return fail(ADI_EINVAL, "u_half and u_curr must be distinct buffers");
    if (adi_status s = check_src(f)) return s;
    if (adi_status s = check_src(f_half)) return s;
    if (adi_status s = check_rec(rec)) return s;
    return w->dtype == ADI_F32 ? do_step_split<float>(w, mode, u_half, u_curr, f, f_half, rec)
                               : do_step_split<double>(w, mode, u_half, u_curr, f, f_half, rec);
}

}  // extern "C"
