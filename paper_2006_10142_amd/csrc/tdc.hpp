// tdc.hpp -- one step of eq. (CN1) with a coefficient that changes in time:
// c^{n+1} multiplies the Laplacian of u^{n+1}, c^{n-1} that of u^{n-1}.  With
// delta = u^{n+1} - 2u^n + u^{n-1}, beta = dt^2/2 and r = beta kappa / h^2,
//     (I - beta K^{n+1} Lap) delta = dt^2 f + 2 r^{n+1} S(u^n) + (r^{n-1} - r^{n+1}) S(u^{n-1}),
// S(v) = v_W + v_E + v_S + v_N - 4 v_C, and the ADI step factors the operator as
// (I - beta K^{n+1} Lxx)(I - beta K^{n+1} Lyy): the x-lines, then the y-lines and
// the update, with the exact two-pass kernels on the coefficient r^{n+1}.  For a
// coefficient constant in time it is the plain step.  Included at the end of
// adiwave.hip.

namespace adw {

// rho = 2 rn S(uc) + (rp - rn) S(up)
template <typename T>
__global__ void __launch_bounds__(256) k_rhs_tdc(const T* __restrict__ uc, const T* __restrict__ up,
                                                 const T* __restrict__ rn, const T* __restrict__ rp,
                                                 T* __restrict__ rho, int nx, int ny)
{
    const long long n = (long long)nx * ny;
    for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < n; p += (long long)gridDim.x * 256) {
        const int j = (int)(p / nx), i = (int)(p - (long long)j * nx);
        auto S = [&](const T* u) {
            const T w_ = i > 0 ? u[p - 1] : T(0), e_ = i < nx - 1 ? u[p + 1] : T(0);
            const T s_ = j > 0 ? u[p - nx] : T(0), n_ = j < ny - 1 ? u[p + nx] : T(0);
            return ((w_ + e_) + (s_ + n_)) - T(4) * u[p];
        };
        const T r1 = rn[p];
        rho[p] = fma_rn(rp[p] - r1, S(up), T(2) * r1 * S(uc));
    }
}

}  // namespace adw

namespace {

template <typename T>
adi_status do_step_tdc(adi_wave_s* w, void** u_prev, void** u_curr, const void* kappa_prev,
                       const void* kappa_next, const adi_source* f, const adi_receivers* rec)
{
    const long long n = (long long)w->nx * w->ny;
    const size_t bytes = (size_t)n * sizeof(T);
    if (!w->r_prev || !w->rho_buf) {
        if (!w->r_prev && hipMalloc(&w->r_prev, bytes) != hipSuccess) {
            (void)hipGetLastError();
            w->r_prev = nullptr;
            return fail(ADI_ENOMEM, "hipMalloc of the previous coefficient failed");
        }
        if (!w->rho_buf && hipMalloc(&w->rho_buf, bytes) != hipSuccess) {
            (void)hipGetLastError();
            w->rho_buf = nullptr;
            return fail(ADI_ENOMEM, "hipMalloc of the right-hand side failed");
        }
        w->bytes += 2 * bytes;
    }
    const double s = w->dt * w->dt / (2.0 * w->h * w->h);
    // r^{n-1}: from kappa_prev, or the handle's current coefficient
    if (kappa_prev) {
        hipLaunchKernelGGL((k_coef<T>), dim3(cr_grid(n)), dim3(256), 0, w->stream, static_cast<const T*>(kappa_prev),
                           T(0), 0, (T)s, static_cast<T*>(w->r_prev), n);
        ADI_LAUNCHED("coef (previous level)");
    } else {
        ADI_HIP(hipMemcpyAsync(w->r_prev, w->r, bytes, hipMemcpyDeviceToDevice, w->stream));
    }
    // r^{n+1} with its x-line pivots and y-chunk planes becomes the handle's coefficient
    if (kappa_next) {
        if (adi_status st = set_coef<T>(w, kappa_next, 0.0, 0, false)) return st;
        // r is no longer measured: the one-pass step stays off until the next set_kappa
        w->fused_ok = 0;
        w->fstep = 0;
    }
    hipLaunchKernelGGL((k_rhs_tdc<T>), dim3(cr_grid(n)), dim3(256), 0, w->stream, static_cast<const T*>(*u_curr),
                       static_cast<const T*>(*u_prev), static_cast<const T*>(w->r),
                       static_cast<const T*>(w->r_prev), static_cast<T*>(w->rho_buf), w->nx, w->ny);
    ADI_LAUNCHED("rhs (time-dependent coefficient)");
    if (f && f->count > 0) {
        hipLaunchKernelGGL((k_cr_sources<T>), dim3(1), dim3(64), 0, w->stream, static_cast<T*>(w->rho_buf), f->idx,
                           static_cast<const T*>(f->amp), f->count, (T)(w->dt * w->dt), n);
        ADI_LAUNCHED("sources");
    }
    if (adi_status st = queue_xsolve<T>(w, w->rho_buf, w->w)) return st;
    YArgs<T> ya = make_y<T>(w, *u_curr, *u_prev, *u_prev, T(2), T(-1));
    const dim3 yg((w->nx + 255) / 256, w->K);
    hipLaunchKernelGGL((k_yreduce<T>), yg, dim3(256), 0, w->stream, ya);
    ADI_LAUNCHED("y_reduce");
    if (!launch_yscan<T>(w->yq, w->nx, ya, w->stream))
        return fail(ADI_EUNSUPPORTED, "no y-interface kernel for this configuration");
    ADI_LAUNCHED("y_scan");
    if (!launch_ysolve<T>(w->M, yg, ya, w->stream))
        return fail(ADI_EUNSUPPORTED, "no y-solve kernel for this chunk size");
    ADI_LAUNCHED("y_solve_update");
    if (rec && rec->count > 0) {
        hipLaunchKernelGGL((k_record<T>), dim3((rec->count + 255) / 256), dim3(256), 0, w->stream,
                           static_cast<const T*>(*u_prev), rec->idx, static_cast<T*>(rec->traces), rec->count, n);
        ADI_LAUNCHED("record");
    }
    std::swap(*u_prev, *u_curr);
    return ADI_OK;
}

}  // namespace

extern "C" {

adi_status adi_wave_step_tdc(adi_wave_t w, void** u_prev, void** u_curr, const void* kappa_prev,
                             const void* kappa_next, const adi_source* f, const adi_receivers* rec)
{
    if (adi_status s = check_handle(w)) return s;
    if (!u_prev || !u_curr || !*u_prev || !*u_curr) return fail(ADI_EINVAL, "null level pointer");
    if (*u_prev == *u_curr) return fail(ADI_EINVAL, "u_prev and u_curr must be distinct buffers");
    if (adi_status s = check_src(f)) return s;
    if (adi_status s = check_rec(rec)) return s;
    return w->dtype == ADI_F32 ? do_step_tdc<float>(w, u_prev, u_curr, kappa_prev, kappa_next, f, rec)
                               : do_step_tdc<double>(w, u_prev, u_curr, kappa_prev, kappa_next, f, rec);
}

}  // extern "C"
