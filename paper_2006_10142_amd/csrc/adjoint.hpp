// adjoint.hpp -- reverse-time adjoint of the ADI run: gradients of a function
// of the receiver traces with respect to the per-node coefficient kappa (and
// the source values).  Included at the end of adiwave.hip.
//
// With A_x = I - beta K Lxx, A_y = I - beta K Lyy and lambda^m = dJ/du^m, step
// k (u^{k-1}, u^k -> u^{k+1}) contributes, backwards in time,
//   nu = A_y^{-T} lambda^{k+1},  mu = A_x^{-T} nu,
//   dJ/dkappa += dt^2 mu Lap(u^k) + beta (mu Lxx w^k + nu Lyy d^k),
//   lambda^k = g^k + 2 lambda^{k+1} - lambda^{k+2} + dt^2 Lap(kappa mu),
// with g^m the direct derivative through the traces of level m.
// A_x = K (K^{-1} - beta Lxx) with a symmetric second factor, hence
//   A_x^{-T} v = R^{-1} A_x^{-1} (R v),   R = diag(r), r = beta kappa / h^2,
// and likewise for A_y: the transposed solves are the forward line solves in
// the other order (y first, then x) on R lambda, divided by r afterwards:
//   z = A_y^{-1} (R lambda^{k+1}),  t = A_x^{-1} z,  nu = z / r,  mu = t / r,
// and dt^2 Lap(kappa mu) = 2 (5-point sum of t - 4 t).  d^k is recovered from
// the stored levels as u^{k+1} - 2u^k + u^{k-1}, and w^k as A_y d^k =
// d^k - r (d^k above + d^k below - 2 d^k) (zero beyond the walls), so that only
// levels are kept.  Levels are checkpointed every K steps by the forward run,
// which takes the handle's step (the one-pass step where it is allowed); each
// segment is recomputed once with the exact two-pass step (its kernels share the
// device with the reverse pass far better than the one-pass step's, which fill
// whole compute units), in reverse segment order, on a second stream into one of
// two halves of the segment storage, so that the recomputation of segment c - 1
// runs while the reverse pass of segment c does (events order them).

namespace adw {

template <typename T>
struct AdjArgs {
    const T* t;      // A_x^{-1} z
    const T* z;      // A_y^{-1} (r lambda^{k+1})
    const T* r;
    const T* lam1;   // lambda^{k+1}
    T* lam2;         // in: lambda^{k+2}; out: lambda^k (without g^k)
    const T* um;     // u^{k-1}
    const T* uk;     // u^k
    const T* up;     // u^{k+1}
    T* grad;         // dJ/dkappa, accumulated
    int nx, ny;
    T c1, c2;        // dt^2 / h^2, beta / h^2
    // point terms of the step (see k_adjoint_points), folded into the same launch:
    const int* rmap;     // per node: first receiver of the node (>= nrec: none)
    const int* rnext;    // per receiver: next receiver of the same node, or -1
    const int* rrow;     // per row: nonzero when a receiver lies in it (rows without skip rmap)
    const T* rvals;      // this step's receiver values (NULL: none)
    const int* sidx;     // source nodes (NULL: no source gradient)
    T* gout;             // dJ/d(source value) of this step
    int nsrc, nrec;
    T tau2;
    long long npts;
};

template <typename T>
__global__ void __launch_bounds__(256) k_adjoint_update(AdjArgs<T> A)
{
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (A.sidx && blockIdx.x == 0 && blockIdx.y == 0) {
        // dJ/d(source value) = tau^2 t / r at the source node (every thread of the block)
        for (int s = threadIdx.x; s < A.nsrc; s += 256) {
            const int id = A.sidx[s];
            A.gout[s] = (id >= 0 && id < A.npts) ? A.tau2 * A.t[id] / A.r[id] : T(0);
        }
    }
    if (i >= A.nx || j >= A.ny) return;
    const int nx = A.nx, ny = A.ny;
    const size_t p = (size_t)j * nx + i;
    auto at = [&](const T* a, int ii, int jj) -> T {
        return (ii >= 0 && ii < nx && jj >= 0 && jj < ny) ? a[(size_t)jj * nx + ii] : T(0);
    };
    auto dlt = [&](int ii, int jj) -> T {   // d^k at (ii, jj), 0 outside the grid
        return (ii >= 0 && ii < nx && jj >= 0 && jj < ny)
                   ? (at(A.up, ii, jj) - T(2) * at(A.uk, ii, jj)) + at(A.um, ii, jj) : T(0);
    };
    auto sydat = [&](int ii) -> T { return (dlt(ii, j - 1) + dlt(ii, j + 1)) - T(2) * dlt(ii, j); };
    auto wat = [&](int ii) -> T {           // w^k = A_y d^k at (ii, j), 0 outside the grid
        return (ii >= 0 && ii < nx) ? dlt(ii, j) - at(A.r, ii, j) * sydat(ii) : T(0);
    };
    const T tc = A.t[p];
    const T s5t = ((at(A.t, i - 1, j) + at(A.t, i + 1, j)) + (at(A.t, i, j - 1) + at(A.t, i, j + 1))) - T(4) * tc;
    const T uc = A.uk[p];
    const T s5u = ((at(A.uk, i - 1, j) + at(A.uk, i + 1, j)) + (at(A.uk, i, j - 1) + at(A.uk, i, j + 1))) - T(4) * uc;
    const T sxw = (wat(i - 1) + wat(i + 1)) - T(2) * wat(i);
    const T syd = sydat(i);
    const T rp = A.r[p];
    const T mu = tc / rp;
    const T nu = A.z[p] / rp;
    A.grad[p] += mu * (A.c1 * s5u + A.c2 * sxw) + nu * (A.c2 * syd);
    T lam = (T(2) * A.lam1[p] - A.lam2[p]) + T(2) * s5t;
    if (A.rvals) {
        // the receivers of this node, in increasing index (the order of k_adjoint_points)
        const int j0 = A.rmap[p];
        for (int j = j0 < A.nrec ? j0 : -1; j >= 0; j = A.rnext[j]) lam += A.rvals[j];
    }
    A.lam2[p] = lam;
}

// The same update with 16 bytes of every field per thread (4 FP32 / 2 FP64 nodes
// of one row; nx a multiple of that, 16-byte aligned fields), rows in XCD bands.  Every load is
// independent of the others; the x-neighbours across a lane's edges come from the
// neighbouring lanes by a wavefront shift, and from memory only at the
// wavefront's two ends.  The receiver map is read only by workgroups whose part of
// the row holds a receiver.  The expressions are those of k_adjoint_update.
template <typename T>
__global__ void __launch_bounds__(256) k_adjoint_update_v(AdjArgs<T> A)
{
    using V = Vec16<T>;
    constexpr int N = V::N;
    using VT = typename V::type;
    const int lane = threadIdx.x & 63;
    const int nx = A.nx, ny = A.ny;
    // work index (row j, column block bx) of this workgroup: the workgroups of one XCD
    // take a contiguous band of rows, so the rows above and below a row are read
    // through the same L2 (the grid is a multiple of 8; workgroups past the last row exit)
    const int gx = (nx / N + 255) / 256;
    const int wk = xcd_band(blockIdx.x);
    const int j = wk / gx, bx = wk - j * gx;
    if (j >= ny) return;
    const int i0 = (bx * 256 + threadIdx.x) * N;
    if (A.sidx && blockIdx.x == 0) {
        for (int s = threadIdx.x; s < A.nsrc; s += 256) {
            const int id = A.sidx[s];
            A.gout[s] = (id >= 0 && id < A.npts) ? A.tau2 * A.t[id] / A.r[id] : T(0);
        }
    }
    const bool in = i0 < nx;
    const bool hn = in && j > 0, hs = in && j + 1 < ny;
    const size_t snx = (size_t)nx;
    const size_t p = (size_t)j * snx + (in ? i0 : 0);
    auto ld = [&](const T* a, size_t q, bool ok, T (&v)[N]) {
        if (ok) V::unpack(*reinterpret_cast<const VT*>(a + q), v);
        else {
#pragma unroll
            for (int e = 0; e < N; ++e) v[e] = T(0);
        }
    };
    T tc[N], tn[N], ts[N], uc[N], un[N], us[N], pc[N], pn[N], ps[N], mc[N], mn[N], ms[N];
    T zc[N], rc[N], l1[N], l2[N], gc[N];
    ld(A.t, p, in, tc); ld(A.t, p - snx, hn, tn); ld(A.t, p + snx, hs, ts);
    ld(A.uk, p, in, uc); ld(A.uk, p - snx, hn, un); ld(A.uk, p + snx, hs, us);
    ld(A.up, p, in, pc); ld(A.up, p - snx, hn, pn); ld(A.up, p + snx, hs, ps);
    ld(A.um, p, in, mc); ld(A.um, p - snx, hn, mn); ld(A.um, p + snx, hs, ms);
    ld(A.z, p, in, zc); ld(A.r, p, in, rc);
    ld(A.lam1, p, in, l1); ld(A.lam2, p, in, l2); ld(A.grad, p, in, gc);
    // d^k of the rows above, at and below, its y second difference, and w^k = A_y d^k
    T syd[N], wc[N];
#pragma unroll
    for (int e = 0; e < N; ++e) {
        const T dn = hn ? (pn[e] - T(2) * un[e]) + mn[e] : T(0);
        const T dc = (pc[e] - T(2) * uc[e]) + mc[e];
        const T ds = hs ? (ps[e] - T(2) * us[e]) + ms[e] : T(0);
        syd[e] = (dn + ds) - T(2) * dc;
        wc[e] = dc - rc[e] * syd[e];
    }
    // values beyond the wavefront's first and last lanes (w^k from the levels there)
    const bool le = lane == 0 && in && i0 > 0, re = lane == 63 && in && i0 + N < nx;
    auto wmem = [&](size_t q) -> T {
        auto d = [&](size_t qq) -> T { return (A.up[qq] - T(2) * A.uk[qq]) + A.um[qq]; };
        const T dc = d(q), dn = hn ? d(q - snx) : T(0), ds = hs ? d(q + snx) : T(0);
        return dc - A.r[q] * ((dn + ds) - T(2) * dc);
    };
    const T tle = le ? A.t[p - 1] : T(0), tre = re ? A.t[p + N] : T(0);
    const T ule = le ? A.uk[p - 1] : T(0), ure = re ? A.uk[p + N] : T(0);
    const T wle = le ? wmem(p - 1) : T(0), wre = re ? wmem(p + N) : T(0);
    const T tl = dpp<kWaveShr1>(tle, tc[N - 1]), tr = dpp<kWaveShl1>(tre, tc[0]);
    const T ul = dpp<kWaveShr1>(ule, uc[N - 1]), ur = dpp<kWaveShl1>(ure, uc[0]);
    const T wl = dpp<kWaveShr1>(wle, wc[N - 1]), wr = dpp<kWaveShl1>(wre, wc[0]);
    const bool row_rec = A.rvals && A.rrow[j] != 0;
    if (!in) return;
    T go[N], lo[N];
#pragma unroll
    for (int e = 0; e < N; ++e) {
        const T tw = e == 0 ? tl : tc[e - 1], te = e == N - 1 ? tr : tc[e + 1];
        const T uw = e == 0 ? ul : uc[e - 1], ue = e == N - 1 ? ur : uc[e + 1];
        const T ww = e == 0 ? wl : wc[e - 1], we = e == N - 1 ? wr : wc[e + 1];
        const T s5t = ((tw + te) + (tn[e] + ts[e])) - T(4) * tc[e];
        const T s5u = ((uw + ue) + (un[e] + us[e])) - T(4) * uc[e];
        const T sxw = (ww + we) - T(2) * wc[e];
        const T mu = tc[e] / rc[e];
        const T nu = zc[e] / rc[e];
        go[e] = gc[e] + (mu * (A.c1 * s5u + A.c2 * sxw) + nu * (A.c2 * syd[e]));
        T lam = (T(2) * l1[e] - l2[e]) + T(2) * s5t;
        if (row_rec) {
            const int j0 = A.rmap[p + e];
            for (int k = j0 < A.nrec ? j0 : -1; k >= 0; k = A.rnext[k]) lam += A.rvals[k];
        }
        lo[e] = lam;
    }
    *reinterpret_cast<VT*>(A.grad + p) = V::pack(go);
    *reinterpret_cast<VT*>(A.lam2 + p) = V::pack(lo);
}

// ---------------------------------------------- transposed x-lines + update --
// t = A_x^{-1} z of one reverse step with the step's update (the expressions of
// k_adjoint_update) folded in, so that t never goes to memory: a line group of TR
// threads (kSeg nodes each, the layout of xsweep.hpp) owns a strip of RS output
// rows and solves the x-lines of rows j0 - 1 .. j0 + RS (the neighbouring strips
// solve the rows above and below again, with the same arithmetic); once the row
// below a row is solved, that row's update runs from registers: t of rows q - 1,
// q, q + 1 (its x-neighbours across segment edges through LDS), z and r of row q
// (the solve's inputs), and u^k, d^k of rows q - 1 .. q + 1 rolled down the strip,
// which give w^k = A_y d^k of row q (its x-neighbours across segment edges from
// the neighbouring lanes, at a wavefront's ends from the levels in memory).
template <typename T, int TR>
struct XUShared {
    T halo[2][2][TR];            // first and last t of every segment, by row parity
    T totf[2][TR / 64][2];       // wavefront totals of the scans (xline_row)
    T totb[2][TR / 64][3];
    int src_pos[kStripSrc];      // sources in the strip's output rows: row offset * 2^16 + column
    int src_k[kStripSrc];        //   and the source's index
    int src_n;                   // count, or -1 when the strip holds more than kStripSrc
};

template <typename T, int TR, bool VEC>
__device__ __forceinline__ void xsolve_update_strip(const XArgs<T>& X, const AdjArgs<T>& A, const int strip,
                                                    const int t, XUShared<T, TR>& sh)
{
    constexpr int E = kSeg;
    const int lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int nx = X.nx, ny = X.ny, nseg = X.nseg;
    const int RS = X.rows_per_strip;
    const int j0 = strip * RS;
    const int j1 = min(j0 + RS, ny);              // output rows [j0, j1)
    const int i0 = E * t;
    const bool act = t < nseg;
    const int L = act ? min(E, nx - i0) : 0;
    const int voff = i0 * (int)sizeof(T);
    const int row_bytes = nx * (int)sizeof(T);
    const long long npts = (long long)nx * ny;
    auto seg = [&](const T* base, int row, T (&v)[E]) {      // this lane's nodes of a row, 0 outside
        const bool in = row >= 0 && row < ny;
        if constexpr (VEC) {
            bload8<T>(buf(base + (size_t)(in ? row : 0) * nx, in ? row_bytes : 0), voff, v);
        } else if (act && in) {
            gload8<T>(base + (size_t)row * nx, i0, nx, v);
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = T(0);
        }
    };
    auto put = [&](T* base, int row, const T (&v)[E]) {
        if constexpr (VEC) bstore8<T>(buf(base + (size_t)row * nx, row_bytes), voff, v);
        else if (act) gstore8<T>(base + (size_t)row * nx, i0, nx, v);
    };
    auto one = [&](const T* base, int row, int col) -> T {   // a single value, 0 outside
        return (act && row >= 0 && row < ny && col >= 0 && col < nx) ? base[(size_t)row * nx + col] : T(0);
    };
    auto dat = [&](int row, int col) -> T {                   // d^k at a node, 0 outside
        return (row >= 0 && row < ny && col >= 0 && col < nx)
                   ? (A.up[(size_t)row * nx + col] - T(2) * A.uk[(size_t)row * nx + col]) + A.um[(size_t)row * nx + col]
                   : T(0);
    };
    auto wmem = [&](int row, int col) -> T {                  // w^k = A_y d^k at a node, 0 outside
        if (col < 0 || col >= nx) return T(0);
        const T dc = dat(row, col);
        return dc - A.r[(size_t)row * nx + col] * ((dat(row - 1, col) + dat(row + 1, col)) - T(2) * dc);
    };

    // sources in the output rows, in source order (wavefront 0 of the group, ballot-compacted)
    if (t < 64) {
        int n = 0;
        for (int base = 0; base < A.nsrc; base += 64) {
            const int k = base + t;
            const int id = (A.sidx && k < A.nsrc) ? A.sidx[k] : -1;
            const int row = (id >= 0 && id < npts) ? id / nx : -1;
            const bool hit = row >= j0 && row < j1;
            const unsigned long long mask = __ballot(hit);
            const int before = __popcll(mask & ((1ull << t) - 1ull));
            if (hit && n + before < kStripSrc) {
                sh.src_pos[n + before] = ((row - j0) << 16) | (id - row * nx);
                sh.src_k[n + before] = k;
            }
            n += __popcll(mask);
        }
        if (t == 0) sh.src_n = n <= kStripSrc ? n : -1;
    }

    // rows q - 1 and q of t, u^k and d^k (rolled down the strip), z and r of row q
    T tm[E], tq[E], ua[E], ub[E], da[E], db[E], zq[E], rq[E];
#pragma unroll
    for (int e = 0; e < E; ++e) { tm[e] = tq[e] = ua[e] = ub[e] = da[e] = db[e] = zq[e] = rq[e] = T(0); }

    // inputs of the first row's solve; each pass requests those of the next row
    // before it solves its own
    auto pivot_in = [&](int row) -> T { return (act && row >= 0 && row < ny) ? X.qin[(size_t)row * nseg + t] : T(0); };
    T zc[E], rc[E];
    seg(X.u, j0 - 1, zc);
    seg(X.r, j0 - 1, rc);
    T qc = pivot_in(j0 - 1);
    for (int j = j0 - 1; j <= j0 + RS; ++j) {
        const int q = j - 1;                       // the row updated in this pass
        const bool upd = q >= j0 && q < j1;
        T zn[E], rn[E];
        const int jn = j < j0 + RS ? j + 1 : -1;   // no row after the strip's last
        seg(X.u, jn, zn);
        seg(X.r, jn, rn);
        const T qn = pivot_in(jn);
        // u^k and d^k of row j, and the update's row q
        T un[E], pn[E], mn[E];
        seg(A.uk, j, un);
        seg(A.up, j, pn);
        seg(A.um, j, mn);
        T l1[E], l2[E], gq[E];
        T uwe = T(0), uee = T(0), wwm = T(0), wem = T(0);
        if (upd) {
            seg(A.lam1, q, l1);
            seg(A.lam2, q, l2);
            seg(A.grad, q, gq);
            uwe = one(A.uk, q, i0 - 1); uee = one(A.uk, q, i0 + L);
            // w^k of row q just beyond the wavefront's first and last lanes
            if (lane == 0) wwm = wmem(q, i0 - 1);
            if (lane == 63) wem = wmem(q, i0 + L);
        }
        // solve row j (rows outside the grid have z = r = 0 and give t = 0)
        T rho[E], tn[E];
#pragma unroll
        for (int e = 0; e < E; ++e) rho[e] = X.rho_scale * zc[e];
        xline_row<T, TR>(rho, rc, qc, L, act, lane, wv, j & 1, sh.totf, sh.totb, []() {}, tn);
        if (act) {
            T last = tn[0];
#pragma unroll
            for (int e = 1; e < E; ++e)
                if (e == L - 1) last = tn[e];
            sh.halo[j & 1][0][t] = tn[0];
            sh.halo[j & 1][1][t] = last;
        }
        T dn[E];
        const bool jin = j >= 0 && j < ny;
#pragma unroll
        for (int e = 0; e < E; ++e) dn[e] = jin ? (pn[e] - T(2) * un[e]) + mn[e] : T(0);
        // w^k = A_y d^k of row q (every lane of the wavefront, so that the lane shifts
        // below read defined values; lanes past the line hold zeros)
        T wq[E], syq[E];
        T wwe = T(0), wee = T(0);
        if (upd) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                syq[e] = (da[e] + dn[e]) - T(2) * db[e];
                wq[e] = db[e] - rq[e] * syq[e];
            }
            wwe = dpp<kWaveShr1>(wwm, wq[E - 1]);
            wee = dpp<kWaveShl1>(wem, wq[0]);
        }
        if (upd && act) {
            // t across the segment edges of row q (written in the previous pass, before
            // this pass's barrier)
            const T tw0 = t > 0 ? sh.halo[q & 1][1][t - 1] : T(0);
            const T teL = t + 1 < nseg ? sh.halo[q & 1][0][t + 1] : T(0);
            const bool row_rec = A.rvals && A.rrow[q] != 0;
            const size_t p0 = (size_t)q * nx + i0;
            T go[E], lo[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const T tw = e == 0 ? tw0 : tq[e - 1], te = e == L - 1 ? teL : (e + 1 < E ? tq[e + 1] : T(0));
                const T uw = e == 0 ? uwe : ub[e - 1], ue = e == L - 1 ? uee : (e + 1 < E ? ub[e + 1] : T(0));
                const T ww = e == 0 ? wwe : wq[e - 1], we = e == L - 1 ? wee : (e + 1 < E ? wq[e + 1] : T(0));
                const T s5t = ((tw + te) + (tm[e] + tn[e])) - T(4) * tq[e];
                const T s5u = ((uw + ue) + (ua[e] + un[e])) - T(4) * ub[e];
                const T sxw = (ww + we) - T(2) * wq[e];
                const T syd = syq[e];
                T g = gq[e], lam = l2[e];
                if (e < L) {
                    const T mu = tq[e] / rq[e];
                    const T nu = zq[e] / rq[e];
                    g = gq[e] + (mu * (A.c1 * s5u + A.c2 * sxw) + nu * (A.c2 * syd));
                    lam = (T(2) * l1[e] - l2[e]) + T(2) * s5t;
                    if (row_rec) {
                        const int k0 = A.rmap[p0 + e];
                        for (int k = k0 < A.nrec ? k0 : -1; k >= 0; k = A.rnext[k]) lam += A.rvals[k];
                    }
                }
                go[e] = g;
                lo[e] = lam;
            }
            put(A.grad, q, go);
            put(A.lam2, q, lo);
            // dJ/d(source value) = tau^2 t / r at the source nodes of row q
            if (A.gout) {
                const int ns = sh.src_n;
                for (int k = 0; k < (ns >= 0 ? ns : A.nsrc); ++k) {
                    int col, kk;
                    if (ns >= 0) {
                        const int pos = sh.src_pos[k];
                        if ((pos >> 16) != q - j0) continue;
                        col = pos & 0xffff;
                        kk = sh.src_k[k];
                    } else {
                        const int id = A.sidx[k];
                        if (id < 0 || id >= npts || id / nx != q) continue;
                        col = id - q * nx;
                        kk = k;
                    }
#pragma unroll
                    for (int e = 0; e < E; ++e)
                        if (i0 + e == col && e < L) A.gout[kk] = A.tau2 * tq[e] / rq[e];
                }
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            tm[e] = tq[e]; tq[e] = tn[e];
            ua[e] = ub[e]; ub[e] = un[e];
            da[e] = db[e]; db[e] = dn[e];
            zq[e] = zc[e]; rq[e] = rc[e];
            zc[e] = zn[e]; rc[e] = rn[e];
        }
        qc = qn;
    }
}

template <typename T, int TR>
__global__ void __launch_bounds__(TR >= 256 ? TR : 256) k_xsolve_update(XArgs<T> X, AdjArgs<T> A)
{
    constexpr int G = (TR >= 256 ? TR : 256) / TR;
    __shared__ XUShared<T, TR> sh[G];
    // sources outside the grid: zero gradient (the strips see only the others)
    if (A.gout && blockIdx.x == 0)
        for (int k = threadIdx.x; k < A.nsrc; k += blockDim.x) {
            const int id = A.sidx[k];
            if (id < 0 || id >= A.npts) A.gout[k] = T(0);
        }
    const int blk = X.xcd ? (int)((blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3)) : (int)blockIdx.x;
    const int strips = (X.ny + X.rows_per_strip - 1) / X.rows_per_strip;
    if (blk * G >= strips) return;
    const int g = __builtin_amdgcn_readfirstlane(threadIdx.x / TR);
    if (X.vec) xsolve_update_strip<T, TR, true>(X, A, blk * G + g, threadIdx.x - g * TR, sh[g]);
    else xsolve_update_strip<T, TR, false>(X, A, blk * G + g, threadIdx.x - g * TR, sh[g]);
}

// The transposed y-lines of one reverse step, z = A_y^{-1} (r lambda), on windows
// (the truncation of the one-pass step, fused.hpp): one thread per (column,
// segment of H rows), the threads of a wavefront on 64 neighbouring columns.  The
// window [j0 - KY, j0 + H + KY) is eliminated downwards from zero carries and
// back-substituted upwards from zero, in registers, and its H central rows are
// written.  Each written row is KY + 1 rows or more from a cut (rows beyond the
// grid have r = 0 and decouple, so the walls need none), so the result differs
// from the full-line solve by at most 2 qs^(KY+1) max|z|, below half an ulp where
// the one-pass bound holds.
template <typename T, int KY, int H>
__global__ void __launch_bounds__(256) k_ysolve_win(const T* __restrict__ lam, const T* __restrict__ r,
                                                   T* __restrict__ z, int nx, int ny)
{
    constexpr int W = H + 2 * KY;
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j0 = (int)(blockIdx.y * 4 + (threadIdx.x >> 6)) * H;
    if (j0 >= ny) return;                                     // no barrier below
    const bool col = i < nx;
    // the whole window is requested before the elimination starts (one memory round
    // trip; the elimination is a chain through the rows)
    T g[W], q[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const int j = j0 - KY + k;
        const bool in = col && j >= 0 && j < ny;
        const size_t p = (size_t)(in ? j : 0) * nx + (col ? i : 0);
        q[k] = in ? r[p] : T(0);
        g[k] = in ? lam[p] : T(0);
    }
    T qc = T(0), gc = T(0);
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const T rr = q[k];
        const T m = pivot_step<T>(rr, qc);
        gc = fma_rn(m, rr * g[k], qc * gc);
        g[k] = gc;
        q[k] = qc;
    }
    T d = T(0);
#pragma unroll
    for (int k = W - 1; k >= KY; --k) {
        d = fma_rn(q[k], d, g[k]);
        const int j = j0 - KY + k;
        if (k < KY + H && col && j < ny) z[(size_t)j * nx + i] = d;
    }
}
constexpr int kYWinRows = 32;   // output rows per thread of k_ysolve_win

// receiver map of the reverse pass: rmap[node] = smallest receiver index at the
// node (rmap filled beforehand with a value above every index, so that a node
// without receivers keeps it), rnext[k] = next receiver at the same node or -1,
// rrow[row] = 1 for every row that holds a receiver (rrow zeroed beforehand)
__global__ void __launch_bounds__(256) k_receiver_map(const int* __restrict__ ridx, int nrec, long long npts,
                                                      int nx, int* rmap, int* rnext, int* rrow)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= nrec) return;
    const int id = ridx[k];
    int nxt = -1;
    if (id >= 0 && id < npts) {
        atomicMin(&rmap[id], k);
        rrow[id / nx] = 1;
        for (int j = k + 1; j < nrec; ++j)
            if (ridx[j] == id) { nxt = j; break; }
    }
    rnext[k] = nxt;
}

// Point terms of one reverse step, one thread per receiver / source index k:
//   receivers: lam[ridx[k]] += vals[k], in increasing k at each node (receivers
//              may share a node: the first receiver of a node adds all of that
//              node's values, in order, so the sums match a sequential loop);
//   sources:   out[k] = tau2 * t[sidx[k]] / r[sidx[k]]  (dJ/d source value).
// Offsets outside [0, npts) are skipped (receivers) or give 0 (sources).
template <typename T>
__global__ void __launch_bounds__(256) k_adjoint_points(T* __restrict__ lam, const int* __restrict__ ridx,
                                                        const T* __restrict__ vals, int nrec,
                                                        const T* __restrict__ t, const T* __restrict__ r,
                                                        const int* __restrict__ sidx, T* __restrict__ out,
                                                        int nsrc, T tau2, long long npts)
{
    __shared__ int itile[256];
    __shared__ T vtile[256];
    const int k = blockIdx.x * 256 + threadIdx.x;
    // every independent load first: the source and receiver indices and values
    const int sid = (out && k < nsrc) ? sidx[k] : -1;
    const bool rec_block = lam && (int)(blockIdx.x * 256) < nrec;   // uniform per block
    const int id = (rec_block && k < nrec) ? ridx[k] : -1;
    const T val = (rec_block && k < nrec) ? vals[k] : T(0);
    bool mine = id >= 0 && id < npts;                        // first receiver of its node
    const T lam0 = mine ? lam[id] : T(0);
    if (out && k < nsrc) out[k] = (sid >= 0 && sid < npts) ? tau2 * t[sid] / r[sid] : T(0);
    if (!rec_block) return;
    T acc = lam0;
    for (int base = 0; base < nrec; base += 256) {
        const bool own = base == (int)(blockIdx.x * 256);       // this block's receivers: registers
        __syncthreads();
        if (base + (int)threadIdx.x < nrec) {
            itile[threadIdx.x] = own ? id : ridx[base + threadIdx.x];
            vtile[threadIdx.x] = own ? val : vals[base + threadIdx.x];
        }
        __syncthreads();
        const int lim = min(256, nrec - base);
        for (int q = 0; mine && q < lim; ++q) {
            if (itile[q] != id) continue;
            if (base + q < k) mine = false;                  // an earlier receiver owns the node
            else acc += vtile[q];
        }
    }
    if (mine) lam[id] = acc;
}

}  // namespace adw

struct adi_adjoint_s {
    int nsteps = 0, K = 0, ncheck = 0;
    unsigned long long record = 0;   // id of the stored forward run (0: none, or invalidated)
    size_t field = 0;            // bytes of one field
    void* ck = nullptr;          // 2 * ncheck fields: (u^{k0-1}, u^{k0}) of every segment
    void* seg = nullptr;         // 2 x K fields, one half per segment parity: levels
                                 // u^{k0+1..k0+K}
    void* work = nullptr;        // 6 fields: forward levels (2; during the reverse pass the
                                 // recomputation's x-sweep output), lambda (2), t, z
    void* rmap = nullptr;        // nx*ny + receiver count + ny ints: receiver map of the reverse pass
    void* ysum = nullptr;        // y-chunk planes and interface values of the recomputation stream
    size_t ck_cap = 0, seg_cap = 0, work_cap = 0, rmap_cap = 0, ysum_cap = 0;
    // the recomputation of segment c - 1 runs on its own stream while the reverse
    // pass of segment c runs on the handle's stream
    hipStream_t rs = nullptr;
    hipEvent_t ev_start = nullptr, ev_rc[2] = {nullptr, nullptr}, ev_rev[2] = {nullptr, nullptr};
};

namespace {

// A coefficient change makes the stored forward run (checkpoints of the old
// trajectory) unusable for a reverse pass.
void adjoint_invalidate(adi_wave_s* w)
{
    if (w->adj) {
        w->adj->record = 0;
        w->adj->nsteps = 0;
    }
}

void adjoint_free(adi_adjoint_s* a)
{
    if (!a) return;
    if (a->rs) (void)hipStreamSynchronize(a->rs);
    if (a->ck) (void)hipFree(a->ck);
    if (a->seg) (void)hipFree(a->seg);
    if (a->work) (void)hipFree(a->work);
    if (a->rmap) (void)hipFree(a->rmap);
    if (a->ysum) (void)hipFree(a->ysum);
    for (hipEvent_t e : {a->ev_start, a->ev_rc[0], a->ev_rc[1], a->ev_rev[0], a->ev_rev[1]})
        if (e) (void)hipEventDestroy(e);
    if (a->rs) (void)hipStreamDestroy(a->rs);
    delete a;
}

// the recomputation stream and its events, created on first use (default priority)
adi_status adjoint_streams(adi_adjoint_s* a)
{
    if (a->rs) return ADI_OK;
    ADI_HIP(hipStreamCreateWithFlags(&a->rs, hipStreamNonBlocking));
    for (hipEvent_t* e : {&a->ev_start, &a->ev_rc[0], &a->ev_rc[1], &a->ev_rev[0], &a->ev_rev[1]})
        ADI_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
    return ADI_OK;
}

adi_status grow(void** p, size_t* cap, size_t need)
{
    if (*cap >= need) return ADI_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    if (hipMalloc(p, need) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(ADI_ENOMEM, "hipMalloc of adjoint storage failed");
    }
    *cap = need;
    return ADI_OK;
}

template <typename T, int TR>
void launch_xsolve1(int grid, const XArgs<T>& a, hipStream_t st)
{
    constexpr int NT = TR >= 256 ? TR : 256;
    hipLaunchKernelGGL((k_xsweep<T, TR, false, false>), dim3(grid), dim3(NT), 0, st, a);
}

// x-line solves of a given field: out = A_x^{-1} rhs
template <typename T>
adi_status queue_xsolve(adi_wave_s* w, const void* rhs, void* out)
{
    XArgs<T> a = make_x<T>(w, rhs, nullptr, 0, T(1));
    a.w = static_cast<T*>(out);
    a.rows_per_strip = w->xp.rs;
    a.xcd = a.rows_per_strip <= kXcdStripRows;
    a.vec = a.vec && aligned16(out);
    const int g = x_groups_per_wg(w->xp.tr);
    const int grid = xsweep_grid(w->ny, w->xp.rs, g);
    switch (w->xp.tr) {
        case 64: launch_xsolve1<T, 64>(grid, a, w->stream); break;
        case 128: launch_xsolve1<T, 128>(grid, a, w->stream); break;
        case 256: launch_xsolve1<T, 256>(grid, a, w->stream); break;
        case 1024: launch_xsolve1<T, 1024>(grid, a, w->stream); break;
        default: return fail(ADI_EUNSUPPORTED, "no x-solve kernel for this plan");
    }
    ADI_LAUNCHED("x_solve");
    return ADI_OK;
}

// the transposed x-lines of z with the update folded in (k_xsolve_update); false
// when the plan's line groups are too wide for it (1024 threads: the registers of
// the update do not fit next to the solve's)
template <typename T>
bool queue_xsolve_update(adi_wave_s* w, const void* z, const AdjArgs<T>& ua)
{
    XArgs<T> a = make_x<T>(w, z, nullptr, 0, T(1));
    a.rows_per_strip = w->xp.rs;
    a.xcd = a.rows_per_strip <= kXcdStripRows;
    a.vec = ((size_t)w->nx * sizeof(T)) % 16 == 0 && aligned16(z) && aligned16(w->r) && aligned16(ua.uk) &&
            aligned16(ua.up) && aligned16(ua.um) && aligned16(ua.lam1) && aligned16(ua.lam2) &&
            aligned16(ua.grad);
    const int grid = xsweep_grid(w->ny, w->xp.rs, x_groups_per_wg(w->xp.tr));
    switch (w->xp.tr) {
        case 64: hipLaunchKernelGGL((k_xsolve_update<T, 64>), dim3(grid), dim3(256), 0, w->stream, a, ua); return true;
        case 128: hipLaunchKernelGGL((k_xsolve_update<T, 128>), dim3(grid), dim3(256), 0, w->stream, a, ua); return true;
        case 256: hipLaunchKernelGGL((k_xsolve_update<T, 256>), dim3(grid), dim3(256), 0, w->stream, a, ua); return true;
    }
    return false;
}

// y-line solves: out = A_y^{-1} (r * rhs)
template <typename T>
adi_status queue_ysolve_scaled(adi_wave_s* w, const void* rhs, void* out)
{
    YArgs<T> ya = make_y<T>(w, nullptr, nullptr, out, T(0), T(0));
    ya.w = static_cast<const T*>(rhs);
    ya.rhs_times_r = 1;
    const dim3 yg((w->nx + 255) / 256, w->K);
    hipLaunchKernelGGL((k_yreduce<T>), yg, dim3(256), 0, w->stream, ya);
    ADI_LAUNCHED("y_reduce (adjoint)");
    if (!launch_yscan<T>(w->yq, w->nx, ya, w->stream))
        return fail(ADI_EUNSUPPORTED, "no y-interface kernel for this configuration");
    ADI_LAUNCHED("y_scan (adjoint)");
    if (!launch_ysolve<T>(w->M, yg, ya, w->stream))
        return fail(ADI_EUNSUPPORTED, "no y-solve kernel for this chunk size");
    ADI_LAUNCHED("y_solve (adjoint)");
    return ADI_OK;
}

adi_source src_at(const adi_source* f, int step0, size_t es)
{
    adi_source s{};
    if (f && f->count > 0) {
        s = *f;
        s.amp = static_cast<const char*>(f->amp) + (size_t)step0 * f->count * es;
    }
    return s;
}

template <typename T>
adi_status adj_forward(adi_wave_s* w, const void* u_prev, const void* u_curr, const adi_source* f,
                       const adi_receivers* rec, int nsteps, int K)
{
    adi_adjoint_s* a = w->adj;
    const size_t F = (size_t)w->nx * w->ny * sizeof(T);
    a->field = F;
    a->nsteps = nsteps;
    a->K = K;
    a->ncheck = (nsteps + K - 1) / K;
    if (adi_status s = grow(&a->ck, &a->ck_cap, 2 * (size_t)a->ncheck * F)) return s;
    if (adi_status s = grow(&a->work, &a->work_cap, 6 * F)) return s;
    char* lev = static_cast<char*>(a->work);
    void* p = lev;
    void* q = lev + F;
    ADI_HIP(hipMemcpyAsync(p, u_prev, F, hipMemcpyDeviceToDevice, w->stream));
    ADI_HIP(hipMemcpyAsync(q, u_curr, F, hipMemcpyDeviceToDevice, w->stream));
    // the handle's step without cyclic reduction: the one-pass step where it is
    // allowed, else the exact two-pass step
    for (int c = 0; c < a->ncheck; ++c) {
        char* ck = static_cast<char*>(a->ck) + 2 * (size_t)c * F;
        ADI_HIP(hipMemcpyAsync(ck, p, F, hipMemcpyDeviceToDevice, w->stream));
        ADI_HIP(hipMemcpyAsync(ck + F, q, F, hipMemcpyDeviceToDevice, w->stream));
        const int n = std::min(K, nsteps - c * K);
        adi_source sc = src_at(f, c * K, sizeof(T));
        adi_receivers rc{};
        if (rec && rec->count > 0) {
            rc = *rec;
            rc.traces = static_cast<char*>(rec->traces) + (size_t)c * K * rec->count * sizeof(T);
        }
        if (adi_status s = do_step<T>(w, &p, &q, f ? &sc : nullptr, rec ? &rc : nullptr, n, kStepNoCr))
            return s;
    }
    return ADI_OK;
}

template <typename T>
adi_status adj_backward(adi_wave_s* w, const adi_source* f, const adi_receivers* rec, const void* grad_traces,
                        void* grad_kappa, void* grad_amp)
{
    adi_adjoint_s* a = w->adj;
    const size_t F = a->field;
    const int S = a->nsteps, K = a->K;
    const long long npts = (long long)w->nx * w->ny;
    if (adi_status s = grow(&a->seg, &a->seg_cap, 2 * (size_t)K * F)) return s;
    if (adi_status s = adjoint_streams(a)) return s;
    // the recomputation's y-chunk workspace: the handle's planes (the static interface
    // coefficients among them) copied, so the two streams never share scratch
    const size_t es = sizeof(T);
    const size_t nsum = (size_t)kSummaryPlanes * w->K * w->nxp, nX = (size_t)w->K * w->nx;
    if (adi_status s = grow(&a->ysum, &a->ysum_cap, (nsum + nX) * es)) return s;
    void* sum2 = a->ysum;
    void* X2 = static_cast<char*>(a->ysum) + nsum * es;
    ADI_HIP(hipMemcpyAsync(sum2, w->sum, nsum * es, hipMemcpyDeviceToDevice, w->stream));
    char* work = static_cast<char*>(a->work);
    T* lam1 = reinterpret_cast<T*>(work + 2 * F);
    T* lam2 = reinterpret_cast<T*>(work + 3 * F);
    T* tt = reinterpret_cast<T*>(work + 4 * F);
    T* zz = reinterpret_cast<T*>(work + 5 * F);
    char* seg = static_cast<char*>(a->seg);
    const int nrec = rec ? rec->count : 0;
    const T* gt = static_cast<const T*>(grad_traces);
    ADI_HIP(hipMemsetAsync(lam1, 0, F, w->stream));
    ADI_HIP(hipMemsetAsync(lam2, 0, F, w->stream));
    ADI_HIP(hipMemsetAsync(grad_kappa, 0, F, w->stream));
    if (nrec > 0) {
        hipLaunchKernelGGL((k_adjoint_points<T>), dim3((nrec + 255) / 256), dim3(256), 0, w->stream, lam1,
                           rec->idx, gt + (size_t)(S - 1) * nrec, nrec, nullptr, nullptr, nullptr, nullptr, 0,
                           T(0), npts);
        ADI_LAUNCHED("adjoint_points");
    }
    const int nsrc = (grad_amp && f) ? f->count : 0;
    const double beta = 0.5 * w->dt * w->dt;
    int* rmap = nullptr;
    int* rnext = nullptr;
    int* rrow = nullptr;
    if (nrec > 0) {
        if (adi_status s = grow(&a->rmap, &a->rmap_cap, ((size_t)npts + nrec + w->ny) * sizeof(int))) return s;
        rmap = static_cast<int*>(a->rmap);
        rnext = rmap + npts;
        rrow = rnext + nrec;
        ADI_HIP(hipMemsetAsync(rmap, 0x7f, (size_t)npts * sizeof(int), w->stream));   // 0x7f7f7f7f: no receiver
        ADI_HIP(hipMemsetAsync(rrow, 0, (size_t)w->ny * sizeof(int), w->stream));
        hipLaunchKernelGGL(k_receiver_map, dim3((nrec + 255) / 256), dim3(256), 0, w->stream, rec->idx, nrec, npts,
                           w->nx, rmap, rnext, rrow);
        ADI_LAUNCHED("receiver_map");
    }
    AdjArgs<T> ua{};
    ua.rmap = rmap;
    ua.rnext = rnext;
    ua.rrow = rrow;
    ua.sidx = nsrc > 0 ? f->idx : nullptr;
    ua.nsrc = nsrc;
    ua.nrec = nrec;
    ua.tau2 = (T)(w->dt * w->dt);
    ua.npts = npts;
    ua.r = static_cast<const T*>(w->r);
    ua.grad = static_cast<T*>(grad_kappa);
    ua.nx = w->nx;
    ua.ny = w->ny;
    ua.c1 = (T)(w->dt * w->dt / (w->h * w->h));
    ua.c2 = (T)(beta / (w->h * w->h));
    const dim3 ug((w->nx + 63) / 64, (w->ny + 3) / 4);
    // the transposed y-lines: on windows (one launch) when the handle takes the FP32
    // one-pass step (whose bound covers their truncation), else the exact chunk solve
    const bool ywin = sizeof(T) == 4 && w->fstep;
    const dim3 ywg((w->nx + 63) / 64, ((w->ny + kYWinRows - 1) / kYWinRows + 3) / 4);
    // 16-byte vectors: whole vectors per row, and every field of the update 16-byte aligned
    // (the handle's and this adjoint's buffers are; the gradient is the caller's)
    constexpr int NV = 16 / (int)sizeof(T);
    const bool vec_upd = w->nx % NV == 0 && aligned16(grad_kappa) && aligned16(w->r) && F % 16 == 0;
    const dim3 ugv((unsigned)((((long long)(w->nx / NV + 255) / 256) * w->ny + 7) / 8 * 8));
    // segment c: levels L[0..n+1] = u^{k0-1} .. u^{k0+n} (L[0], L[1] the checkpoint,
    // the others in half c % 2 of the segment storage)
    auto lev = [&](int c, int m) -> void* {
        if (m < 2) return static_cast<char*>(a->ck) + (2 * (size_t)c + m) * F;
        return seg + ((size_t)K * (c & 1) + (m - 2)) * F;
    };
    // recompute segment c on the recomputation stream with the exact two-pass step
    // (the levels are those of the forward run bit for bit when it took that step;
    // after one-pass steps they differ by at most that step's bound, half an ulp per
    // step)
    auto recompute = [&](int c) -> adi_status {
        const int k0 = 1 + c * K;
        const int n = std::min(K, S - c * K);
        hipStream_t s1 = w->stream;
        void *wkeep = w->w, *skeep = w->sum, *xkeep = w->X;
        w->stream = a->rs;
        w->sum = sum2;
        w->X = X2;
        w->w = work;                             // the x-sweep's output (not kept)
        adi_status s = ADI_OK;
        for (int m = 0; m < n && s == ADI_OK; ++m) {
            adi_source sc = src_at(f, k0 - 1 + m, sizeof(T));
            s = queue_solve<T>(w, lev(c, m + 1), lev(c, m), lev(c, m + 2), T(2), T(-1), f ? &sc : nullptr, 0,
                               T(1), nullptr);
        }
        w->stream = s1;
        w->w = wkeep;
        w->sum = skeep;
        w->X = xkeep;
        return s;
    };
    // the recomputation stream starts after everything queued so far (the checkpoints,
    // the copy of the planes); segment c - 1 is recomputed into the half that segment
    // c + 1 used, once the reverse pass of c + 1 is done with it
    ADI_HIP(hipEventRecord(a->ev_start, w->stream));
    ADI_HIP(hipStreamWaitEvent(a->rs, a->ev_start, 0));
    const int last = a->ncheck - 1;
    if (adi_status s = recompute(last)) return s;
    ADI_HIP(hipEventRecord(a->ev_rc[last & 1], a->rs));
    for (int c = last; c >= 0; --c) {
        if (c >= 1) {
            if (c + 1 <= last) ADI_HIP(hipStreamWaitEvent(a->rs, a->ev_rev[(c + 1) & 1], 0));
            if (adi_status s = recompute(c - 1)) return s;
            ADI_HIP(hipEventRecord(a->ev_rc[(c - 1) & 1], a->rs));
        }
        ADI_HIP(hipStreamWaitEvent(w->stream, a->ev_rc[c & 1], 0));
        const int k0 = 1 + c * K;
        const int n = std::min(K, S - c * K);
        for (int m = n - 1; m >= 0; --m) {
            const int k = k0 + m;
            bool ydone = false;
            if constexpr (sizeof(T) == 4) {
                if (ywin) {
                    hipLaunchKernelGGL((k_ysolve_win<T, kFuKy, kYWinRows>), ywg, dim3(256), 0, w->stream, lam1,
                                       static_cast<const T*>(w->r), zz, w->nx, w->ny);
                    ADI_LAUNCHED("y_solve windows (adjoint)");
                    ydone = true;
                }
            }
            if (!ydone)
                if (adi_status s = queue_ysolve_scaled<T>(w, lam1, zz)) return s;
            ua.t = tt; ua.z = zz; ua.lam1 = lam1; ua.lam2 = lam2;
            ua.um = static_cast<const T*>(lev(c, m));
            ua.uk = static_cast<const T*>(lev(c, m + 1));
            ua.up = static_cast<const T*>(lev(c, m + 2));
            ua.rvals = (k >= 2 && nrec > 0) ? gt + (size_t)(k - 2) * nrec : nullptr;
            ua.gout = nsrc > 0 ? static_cast<T*>(grad_amp) + (size_t)(k - 1) * nsrc : nullptr;
            if (queue_xsolve_update<T>(w, zz, ua)) {
                ADI_LAUNCHED("x_solve + adjoint_update");
            } else {
                if (adi_status s = queue_xsolve<T>(w, zz, tt)) return s;
                if (vec_upd) hipLaunchKernelGGL((k_adjoint_update_v<T>), ugv, dim3(256), 0, w->stream, ua);
                else hipLaunchKernelGGL((k_adjoint_update<T>), ug, dim3(256), 0, w->stream, ua);
                ADI_LAUNCHED("adjoint_update");
            }
            std::swap(lam1, lam2);
        }
        ADI_HIP(hipEventRecord(a->ev_rev[c & 1], w->stream));
    }
    return ADI_OK;
}

}  // namespace

extern "C" {

adi_status adi_adjoint_forward(adi_wave_t w, const void* u_prev, const void* u_curr, const adi_source* f,
                               const adi_receivers* rec, int nsteps, int checkpoint_every,
                               unsigned long long* record)
{
    if (record) *record = 0;
    if (adi_status s = check_handle(w)) return s;
    if (!u_prev || !u_curr) return fail(ADI_EINVAL, "null level pointer");
    if (nsteps < 1) return fail(ADI_EINVAL, "nsteps must be >= 1");
    if (checkpoint_every < 1) return fail(ADI_EINVAL, "checkpoint_every must be >= 1");
    if (adi_status s = check_src(f)) return s;
    if (adi_status s = check_rec(rec)) return s;
    if (!w->adj) w->adj = new adi_adjoint_s();
    w->adj->nsteps = 0;
    w->adj->record = 0;
    adi_status s = w->dtype == ADI_F32
                       ? adj_forward<float>(w, u_prev, u_curr, f, rec, nsteps, checkpoint_every)
                       : adj_forward<double>(w, u_prev, u_curr, f, rec, nsteps, checkpoint_every);
    if (s != ADI_OK) {
        w->adj->nsteps = 0;
        return s;
    }
    w->adj->record = ++w->gen;
    if (record) *record = w->adj->record;
    return ADI_OK;
}

adi_status adi_adjoint_backward(adi_wave_t w, unsigned long long record, const adi_source* f,
                                const adi_receivers* rec, const void* grad_traces, void* grad_kappa,
                                void* grad_amp)
{
    if (adi_status s = check_handle(w)) return s;
    if (!w->adj || w->adj->record == 0 || w->adj->nsteps < 1)
        return fail(ADI_EINVAL, "no forward record: run adi_adjoint_forward first (a coefficient "
                                "change discards the stored forward run)");
    if (record != 0 && record != w->adj->record)
        return fail(ADI_EINVAL, "the forward record was replaced by a later adi_adjoint_forward "
                                "on this handle");
    if (!grad_kappa) return fail(ADI_EINVAL, "grad_kappa is null");
    if (adi_status s = check_src(f)) return s;
    if (adi_status s = check_rec(rec)) return s;
    if (rec && rec->count > 0 && !grad_traces) return fail(ADI_EINVAL, "grad_traces is null");
    return w->dtype == ADI_F32 ? adj_backward<float>(w, f, rec, grad_traces, grad_kappa, grad_amp)
                               : adj_backward<double>(w, f, rec, grad_traces, grad_kappa, grad_amp);
}

}  // extern "C"
