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
// maps across its segments: DPP row shifts / broadcasts inside a wavefront and
// one LDS exchange of wavefront totals (one barrier per row) -- the Thomas
// solution up to rounding.
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
// A 32-bit half whose `old` is a known 0 under full row and bank masks is moved
// with the bound control set instead: lanes without a source then read 0 from the
// hardware, and no register has to be filled with the old value first (the 0
// identity, and the low word of 1.0, cost no instruction).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp_half(int old, int src)
{
    if (ROWMASK == 0xf && __builtin_constant_p(old) && old == 0)
        return __builtin_amdgcn_update_dpp(0, src, CTRL, 0xf, 0xf, true);
    return __builtin_amdgcn_update_dpp(old, src, CTRL, ROWMASK, 0xf, false);
}
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ double dpp(double old, double src)
{
    const long long o = __builtin_bit_cast(long long, old), s = __builtin_bit_cast(long long, src);
    const int lo = dpp_half<CTRL, ROWMASK>((int)o, (int)s);
    const int hi = dpp_half<CTRL, ROWMASK>((int)(o >> 32), (int)(s >> 32));
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

template <int CTRL, int ROWMASK, typename T>
__device__ __forceinline__ void compose3_dpp(T& a0, T& a1, T& b)
{
    const T x0 = dpp<CTRL, ROWMASK>(T(0), a0);
    const T x1 = dpp<CTRL, ROWMASK>(T(0), a1);
    const T b2 = dpp<CTRL, ROWMASK>(T(1), b);
    a0 = fma_rn(b, x0, a0);
    a1 = fma_rn(b, x1, a1);
    b = b * b2;
}

// Wavefront scans of affine maps with each DPP lane move folded into the
// composing multiply-add / multiply: a lane whose source lane does not exist (or
// lies in a row outside the mask) is left as it is, which is composition with the
// identity map, so the results are those of wave_scan_fwd / row_scan_bwd bit for
// bit (the same fused roundings) in a third of the instructions.  A DPP read of a
// register written by the previous VALU instruction needs two wait states: the
// s_nop before, between and after the steps provide them.
#define ADW_FU_STEP(CTRL, MASK) \
    "v_fmac_f32_dpp %0, %0, %1 " CTRL " row_mask:" MASK " bank_mask:0xf\n\t" \
    "v_mul_f32_dpp %1, %1, %1 " CTRL " row_mask:" MASK " bank_mask:0xf\n\t" \
    "s_nop 0\n\t"

// inclusive prefix (lanes 0..l) over the wavefront
__device__ __forceinline__ void fu_scan_fwd(float& a, float& b)
{
    asm volatile("s_nop 1\n\t"
                 ADW_FU_STEP("row_shr:1", "0xf") ADW_FU_STEP("row_shr:2", "0xf")
                 ADW_FU_STEP("row_shr:4", "0xf") ADW_FU_STEP("row_shr:8", "0xf")
                 ADW_FU_STEP("row_bcast:15", "0xa") ADW_FU_STEP("row_bcast:31", "0xc")
                 "s_nop 1"
                 : "+v"(a), "+v"(b));
}

// inclusive suffix over each row of 16 lanes (lanes l..16k+15)
__device__ __forceinline__ void fu_row_scan_bwd(float& a, float& b)
{
    asm volatile("s_nop 1\n\t"
                 ADW_FU_STEP("row_shl:1", "0xf") ADW_FU_STEP("row_shl:2", "0xf")
                 ADW_FU_STEP("row_shl:4", "0xf") ADW_FU_STEP("row_shl:8", "0xf")
                 "s_nop 1"
                 : "+v"(a), "+v"(b));
}
#define ADW_FU_STEP3(CTRL) \
    "v_fmac_f32_dpp %0, %0, %2 " CTRL " row_mask:0xf bank_mask:0xf\n\t" \
    "v_fmac_f32_dpp %1, %1, %2 " CTRL " row_mask:0xf bank_mask:0xf\n\t" \
    "v_mul_f32_dpp %2, %2, %2 " CTRL " row_mask:0xf bank_mask:0xf\n\t"

// inclusive suffix over each row of 16 lanes of three-component maps (a0 + a1 C, b):
// between a register's write and its next DPP read stand the two other
// components' instructions, the two wait states needed
__device__ __forceinline__ void fu_row_scan_bwd3(float& a0, float& a1, float& b)
{
    asm volatile("s_nop 1\n\t"
                 ADW_FU_STEP3("row_shl:1") ADW_FU_STEP3("row_shl:2")
                 ADW_FU_STEP3("row_shl:4") ADW_FU_STEP3("row_shl:8")
                 "s_nop 1"
                 : "+v"(a0), "+v"(a1), "+v"(b));
}
#undef ADW_FU_STEP3
#undef ADW_FU_STEP

// prefix over each row of 16 lanes (lanes 16k..l)
template <typename T>
__device__ __forceinline__ void row_scan_fwd(T& a, T& b)
{
    compose_dpp<kRowShr + 1, 0xf>(a, b);
    compose_dpp<kRowShr + 2, 0xf>(a, b);
    compose_dpp<kRowShr + 4, 0xf>(a, b);
    compose_dpp<kRowShr + 8, 0xf>(a, b);
}
// suffix over each row of 16 lanes (lanes l..16k+15)
template <typename T>
__device__ __forceinline__ void row_scan_bwd(T& a, T& b)
{
    compose_dpp<kRowShl + 1, 0xf>(a, b);
    compose_dpp<kRowShl + 2, 0xf>(a, b);
    compose_dpp<kRowShl + 4, 0xf>(a, b);
    compose_dpp<kRowShl + 8, 0xf>(a, b);
}

// inclusive prefix (lanes 0..l) over the wavefront
template <typename T>
__device__ __forceinline__ void wave_scan_fwd(T& a, T& b)
{
    if constexpr (sizeof(T) == 4) {
        fu_scan_fwd(a, b);
    } else {
        row_scan_fwd(a, b);
        compose_dpp<kRowBcast15, 0xa>(a, b);
        compose_dpp<kRowBcast31, 0xc>(a, b);
    }
}

// inclusive suffix (lanes l..63) of three-component maps (a0 + a1 C, b)
template <typename T>
__device__ __forceinline__ void wave_scan_bwd3(T& a0, T& a1, T& b, int lane)
{
    if constexpr (sizeof(T) == 4) {
        fu_row_scan_bwd3(a0, a1, b);
    } else {
        compose3_dpp<kRowShl + 1, 0xf>(a0, a1, b);
        compose3_dpp<kRowShl + 2, 0xf>(a0, a1, b);
        compose3_dpp<kRowShl + 4, 0xf>(a0, a1, b);
        compose3_dpp<kRowShl + 8, 0xf>(a0, a1, b);
    }
    const T p16 = readlane(a0, 16), q16 = readlane(a1, 16), b16 = readlane(b, 16);
    const T p32 = readlane(a0, 32), q32 = readlane(a1, 32), b32 = readlane(b, 32);
    const T p48 = readlane(a0, 48), q48 = readlane(a1, 48), b48 = readlane(b, 48);
    const T p23 = fma_rn(b32, p48, p32), q23 = fma_rn(b32, q48, q32), b23 = b32 * b48;   // rows 2,3
    const T p13 = fma_rn(b16, p23, p16), q13 = fma_rn(b16, q23, q16), b13 = b16 * b23;   // rows 1..3
    T cp = T(0), cq = T(0), cb = T(1);
    if (lane < 16) { cp = p13; cq = q13; cb = b13; }
    else if (lane < 32) { cp = p23; cq = q23; cb = b23; }
    else if (lane < 48) { cp = p48; cq = q48; cb = b48; }
    a0 = fma_rn(b, cp, a0);
    a1 = fma_rn(b, cq, a1);
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
    int xcd;             // strips in XCD bands (short strips, see k_xsweep)
    int vec;             // rows are 16-byte aligned and nx % 8 == 0
    T rho_scale;         // 1 for a step, 1/2 for the ghost start
    T tau2;              // dt^2
    int nsrc;            // point sources of this step
    const int* src_idx;
    const T* src_amp;    // nsrc values of f
    // fused y-chunk elimination: a strip is a whole number of y-chunks of M rows
    T* sum;              // summary planes (blocked by 16 columns, see kernels.hpp)
    int K, M, nxp;
    // receivers of the previous step, sampled from u (see rec_tap)
    int nrec;
    const int* rec_idx;
    T* rec_out;
};

constexpr int kSeg = 8;   // nodes per x-line segment (one segment per thread)
constexpr int kPB = 16;   // column block width of the y-chunk summary planes

// pivot entering every segment of SEG nodes of every row (SEG = kSeg: the x-sweep's
// segments; 2: the lanes of the FP64 one-pass strips): one thread per row, sequential
template <typename T, int SEG = kSeg>
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
        for (int e = 0; e < SEG; ++e) {
            const int i = SEG * s + e;
            if (i < nx) (void)pivot_step<T>(rr[i], q);
        }
    }
}

// ---------------------------------------------------------- buffer I/O ----
// Rows are read and written through buffer resources whose size is the row's
// byte length (0 for a row outside the grid): the hardware range check returns
// zero for loads past the end and drops such stores, so the accesses need no
// branches and the compiler can count outstanding loads exactly (which keeps
// the row-ahead prefetch in flight across the solve of the current row).
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kBufWord3 = 0x00020000;   // 32-bit data format, gfx9 family

// base and nbytes must be the same in every lane of the wavefront (they are
// moved to scalar registers, so the compiler needs no per-lane loop)
template <typename T>
__device__ __forceinline__ rsrc_t buf(const T* base, int nbytes)
{
    const unsigned long long a = reinterpret_cast<unsigned long long>(base);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
    T* p = reinterpret_cast<T*>(((unsigned long long)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, __builtin_amdgcn_readfirstlane(nbytes), kBufWord3);
}

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
// (whole vectors are bit-cast: a bit cast of a single vector element is not
// compiled correctly by this toolchain)

// 8 consecutive values at byte offset voff with 16-byte accesses.  The row is
// 16-byte aligned and its byte length a multiple of 16, so every access is
// wholly inside or wholly outside the range.
template <typename T>
__device__ __forceinline__ void bload8(rsrc_t rs, int voff, T (&v)[kSeg])
{
    if constexpr (sizeof(T) == 4) {
        const f32x4 x = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, 0, 0));
        const f32x4 y = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff + 16, 0, 0));
        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
        v[4] = y.x; v[5] = y.y; v[6] = y.z; v[7] = y.w;
    } else {
#pragma unroll
        for (int h = 0; h < kSeg / 2; ++h) {
            const f64x2 x = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(rs, voff + 16 * h, 0, 0));
            v[2 * h] = x.x;
            v[2 * h + 1] = x.y;
        }
    }
}

template <typename T>
__device__ __forceinline__ void bstore8(rsrc_t rs, int voff, const T (&v)[kSeg])
{
    if constexpr (sizeof(T) == 4) {
        const f32x4 x = {v[0], v[1], v[2], v[3]};
        const f32x4 y = {v[4], v[5], v[6], v[7]};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(i32x4, x), rs, voff, 0, 0);
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(i32x4, y), rs, voff + 16, 0, 0);
    } else {
#pragma unroll
        for (int h = 0; h < kSeg / 2; ++h) {
            const f64x2 x = {v[2 * h], v[2 * h + 1]};
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(i32x4, x), rs, voff + 16 * h, 0, 0);
        }
    }
}

// Rows without that alignment: per-value global accesses guarded by the row end.
template <typename T>
__device__ __forceinline__ void gload8(const T* __restrict__ row, int i0, int nx, T (&v)[kSeg])
{
#pragma unroll
    for (int e = 0; e < kSeg; ++e) v[e] = (i0 + e < nx) ? row[i0 + e] : T(0);
}
template <typename T>
__device__ __forceinline__ void gstore8(T* __restrict__ row, int i0, int nx, const T (&v)[kSeg])
{
#pragma unroll
    for (int e = 0; e < kSeg; ++e)
        if (i0 + e < nx) row[i0 + e] = v[e];
}

template <typename T>
__device__ __forceinline__ T bload1(rsrc_t rs, int voff)
{
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, 0, 0));
    else
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, 0, 0));
}

// One row of x-lines solved on chip by a line group of TR threads (kSeg nodes each,
// the segment layout above): the local elimination of every segment from its entry
// pivot qc, both affine scans across the line with one workgroup barrier (totals
// of the wavefronts in totf / totb, parity par), and the back substitution into
// wout.  mid() runs after the barrier and before the back substitution (the FP64
// line groups of 1024 threads request their next row of r there).  Every thread of
// the workgroup must call this the same number of times.
template <typename T, int TR, class Mid>
__device__ __forceinline__ void xline_row(const T (&rho)[kSeg], const T (&rc)[kSeg], const T qc, const int L,
                                          const bool act, const int lane, const int wv, const int par,
                                          T (&totf)[2][TR / 64][2], T (&totb)[2][TR / 64][3], Mid&& mid,
                                          T (&wout)[kSeg])
{
    constexpr int E = kSeg;
    constexpr int NW = TR / 64;
    // local elimination of the segment from its entry pivot.  Nodes past the
    // end of the line (e >= L) have r = 0 and rho = 0 (zero-filled loads): they
    // get m = 1, q = 0, G = 0 and add nothing to the segment's maps, so no
    // branch is needed.  A lane without nodes keeps the identity map (0, 1).
    // (the running products of q are not kept per node: the back substitution forms
    // them again, with the same multiplications in the same order, which keeps the
    // FP64 line group of 1024 threads within its 128 registers)
    T Ge[E], qe[E];
    T fG, fQ, H, Ev;
    {
        T q = qc, Gv = T(0), Qv = T(1), h = T(0), ee = T(0);
        T QL = T(1);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const T m = pivot_step<T>(rc[e], q);
            const T P = Qv;                       // prod of q before node e
            Gv = fma_rn(m, rho[e], q * Gv);
            Qv = q * Qv;
            h = fma_rn(P, Gv, h);
            ee = fma_rn(P, Qv, ee);
            Ge[e] = Gv;
            qe[e] = q;
            if (e == L - 1) QL = Qv;
        }
        fG = Gv; fQ = act ? Qv : T(1); H = h; Ev = ee;
        if (L < E) {                              // partial segment: carry the last node's map
#pragma unroll
            for (int e = 0; e < E; ++e)
                if (e == L - 1) fG = Ge[e];
            fQ = QL;
        }
    }

    // Both scans across the line with one workgroup barrier.  The forward maps
    // (g_out = fG + fQ g_in) are scanned inside the wavefront; the value C
    // entering the wavefront is not known yet, so each lane's backward map
    // a = H + Ev g_in = (H + Ev xa) + (Ev xb) C is scanned with C symbolic
    // (components a0, a1).  After the barrier every wavefront combines the
    // totals of all wavefronts: the carries C_k of every wavefront, and from
    // them the backward totals (a0 + a1 C_k, b) and the value D below its last
    // lane.
    T gin, dbelow;
    {
        T a = fG, b = fQ;
        wave_scan_fwd(a, b);
        const T xa = dpp<kWaveShr1>(T(0), a);
        const T xb = dpp<kWaveShr1>(T(1), b);
        T a0 = fma_rn(Ev, xa, H), a1 = Ev * xb, bb = fQ;
        if (!act) { a0 = T(0); a1 = T(0); bb = T(1); }
        wave_scan_bwd3(a0, a1, bb, lane);
        const T ya0 = dpp<kWaveShl1>(T(0), a0);
        const T ya1 = dpp<kWaveShl1>(T(0), a1);
        const T yb = dpp<kWaveShl1>(T(1), bb);
        if constexpr (NW > 1) {
            if (lane == 63) { totf[par][wv][0] = a; totf[par][wv][1] = b; }
            if (lane == 0) { totb[par][wv][0] = a0; totb[par][wv][1] = a1; totb[par][wv][2] = bb; }
        }
        __syncthreads();
        T C = T(0), D = T(0);
        if constexpr (NW > 1) {
            const int k = lane < NW ? lane : 0;
            T fa = (lane < NW) ? totf[par][k][0] : T(0);
            T fb = (lane < NW) ? totf[par][k][1] : T(1);
            row_scan_fwd(fa, fb);                        // lane k: waves 0..k
            const T Ck = dpp<kRowShr + 1, 0xf>(T(0), fa);  // lane k: value entering wave k
            T ta = T(0), tb = T(1);
            if (lane < NW) {
                ta = fma_rn(totb[par][k][1], Ck, totb[par][k][0]);
                tb = totb[par][k][2];
            }
            row_scan_bwd(ta, tb);                        // lane k: waves k..NW-1
            C = readlane(Ck, __builtin_amdgcn_readfirstlane(wv));
            D = (wv + 1 < NW) ? readlane(ta, __builtin_amdgcn_readfirstlane(wv + 1)) : T(0);
        }
        gin = fma_rn(xb, C, xa);
        dbelow = fma_rn(yb, D, fma_rn(ya1, C, ya0));
    }

    mid();

    // back substitution (tail nodes give 0 and feed q = 0 into the last node)
    {
        T Qv = T(1);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            Qv = qe[e] * Qv;
            Ge[e] = fma_rn(Qv, gin, Ge[e]);
        }
        T x = dbelow;
#pragma unroll
        for (int e = E - 1; e >= 0; --e) {
            x = fma_rn(qe[e], x, Ge[e]);
            wout[e] = x;
        }
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
constexpr int kStripSrc = 32;   // point sources staged per strip (more: read per row)

// FP64 line groups of 1024 threads keep the row above the one being solved (u^n,
// row j-1) in LDS instead of registers, and request the next row of r only after
// the scans: with both in registers the group needs more than the 128 VGPRs a
// 1024-thread workgroup allows, and the spills went to scratch memory (twice the
// kernel's algorithmic traffic).  Each thread writes and reads only its own LDS
// slots, so no barrier is involved.
template <typename T, int TR>
constexpr bool kUmLds = sizeof(T) == 8 && TR >= 1024;

template <typename T, int TR, bool FUSE>
struct XShared {
    T um[kUmLds<T, TR> ? kSeg * TR : 1];     // row j-1 of u^n per lane (see kUmLds)
    T halo[2][2][TR];                        // segment edges of two rows: [row parity][first/last][seg]
    T totf[2][TR / 64][2];                   // wavefront totals by row parity: forward (a, b)
    T totb[2][TR / 64][3];                   //   and backward (a0, a1, b)
    T y[FUSE ? 4 * kSeg * TR : 1];           // fused y-chunk state per column
    T src_add[kStripSrc];                    // sources of the strip, in source order:
    int src_pos[kStripSrc];                  //   value added to rho, row offset * 2^16 + column
    int src_n;                               // count, or -1 when the strip has more than kStripSrc
};

// Stage the point sources that fall in rows [j0, j0 + RS) into LDS, in source
// order (wavefront 0, 64 sources per pass, ballot-compacted), so that the row
// loop reads them from LDS instead of global memory.
template <typename T, int TR, bool FUSE>
__device__ __forceinline__ void stage_sources(const XArgs<T>& A, int j0, int RS, int t,
                                              XShared<T, TR, FUSE>& sh)
{
    if (t >= 64) return;
    int n = 0;
    for (int base = 0; base < A.nsrc; base += 64) {
        const int q = base + t;
        int id = -1;
        T amp = T(0);
        if (q < A.nsrc) { id = A.src_idx[q]; amp = A.src_amp[q]; }
        const long long npts = (long long)A.nx * A.ny;
        const int row = (id >= 0 && id < npts) ? id / A.nx : -1;
        const bool hit = row >= j0 && row < j0 + RS;
        const unsigned long long mask = __ballot(hit);
        const int before = __popcll(mask & ((1ull << t) - 1ull));
        if (hit && n + before < kStripSrc) {
            sh.src_add[n + before] = A.rho_scale * A.tau2 * amp;
            sh.src_pos[n + before] = ((row - j0) << 16) | (id - row * A.nx);
        }
        n += __popcll(mask);
    }
    if (t == 0) sh.src_n = n <= kStripSrc ? n : -1;
}

// One strip (rows_per_strip rows from strip * rows_per_strip) of one line group.
// Every thread of the workgroup must call this with the same rows_per_strip
// (it synchronises the workgroup twice per row).
// STENCIL = false: the right-hand side of row j is rho_scale * (row j of A.u)
// instead of the 5-point assembly (line solves of a given field).
template <typename T, int TR, bool FUSE, bool STENCIL, bool VEC>
__device__ __forceinline__ void xsweep_strip_impl(const XArgs<T>& A, const int strip, const int t,
                                                  XShared<T, TR, FUSE>& sh)
{
    constexpr int E = kSeg;
    constexpr int NW = TR / 64;
    auto& s_halo = sh.halo;
    const int lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int nx = A.nx, ny = A.ny, nseg = A.nseg;
    const int RS = A.rows_per_strip;
    const int j0 = strip * RS;
    const int i0 = E * t;
    const bool act = t < nseg;
    const int L = act ? min(E, nx - i0) : 0;

    // rolling rows of u^n (j-1 .. j+2), r and the entry pivots (j, j+1)
    T ua[E], ub[E], uc0[E], ud[E];
    T ra[E], rb[E];
    T qa = T(0), qb = T(0);

    const int voff = i0 * (int)sizeof(T);            // this lane's byte offset in a row
    const int row_bytes = nx * (int)sizeof(T);
    auto zero8 = [&](T (&v)[E]) {
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = T(0);
    };
    auto load_u = [&](int row, T (&v)[E]) {
        const bool in = row >= 0 && row < ny;
        if constexpr (VEC) {
            bload8<T>(buf(A.u + (size_t)(in ? row : 0) * nx, in ? row_bytes : 0), voff, v);
        } else {
            if (act && in) gload8<T>(A.u + (size_t)row * nx, i0, nx, v);
            else zero8(v);
        }
    };
    auto load_rq = [&](int row, T (&v)[E], T& q) {
        const bool in = row >= 0 && row < ny;
        if constexpr (VEC) {
            bload8<T>(buf(A.r + (size_t)(in ? row : 0) * nx, in ? row_bytes : 0), voff, v);
            q = bload1<T>(buf(A.qin + (size_t)(in ? row : 0) * nseg, in ? nseg * (int)sizeof(T) : 0),
                          t * (int)sizeof(T));
        } else if (act && in) {
            gload8<T>(A.r + (size_t)row * nx, i0, nx, v);
            q = A.qin[(size_t)row * nseg + t];
        } else {
            zero8(v);
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

    if constexpr (STENCIL) stage_sources<T, TR, FUSE>(A, j0, RS, t, sh);
    load_u(j0 - 1, ua);
    if constexpr (kUmLds<T, TR>) {
#pragma unroll
        for (int e = 0; e < E; ++e) sh.um[e * TR + t] = ua[e];
    }
    load_u(j0, ub);
    load_u(j0 + 1, uc0);
    load_rq(j0, ra, qa);
    put_halo(j0, ub);
    __syncthreads();

    // Row j = j0 + it.  um, uc, u1 hold rows j-1, j, j+1; u2 receives row j+2.
    // rc, qc: row j; rn, qn receive row j+1.
    auto row = [&](const int it, T (&um)[E], T (&uc)[E], T (&u1)[E], T (&u2)[E], T (&rc)[E], T (&rn)[E],
                   T& qc, T& qn) {
        const int j = j0 + it;
        const bool live = j < ny;
        // prefetch
        load_u(live ? j + 2 : -1, u2);
        // (FP64 line groups of 1024 threads request row j+1 of r after the scans
        // instead, where fewer registers are live: see kUmLds)
        if constexpr (!kUmLds<T, TR>) load_rq(live ? j + 1 : -1, rn, qn);
        // edges of row j+1 (resident since the previous row) for the next row's stencil;
        // the other parity buffer is read below, and row j-1's readers passed a barrier
        if (live && j + 1 < ny) put_halo(j + 1, u1);

        // right-hand side of row j
        T rho[E];
        {
            const int p = j & 1;
            const T west0 = (act && t > 0) ? s_halo[p][1][t - 1] : T(0);
            const T eastL = (t + 1 < nseg) ? s_halo[p][0][t + 1] : T(0);
            // rho_scale * 2 r x == (2 rho_scale) * (r x) exactly: 2 and rho_scale
            // (1 or 1/2) are powers of two
            const T s2 = T(2) * A.rho_scale;
            T umv[E];
#pragma unroll
            for (int e = 0; e < E; ++e) umv[e] = kUmLds<T, TR> ? sh.um[e * TR + t] : um[e];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if constexpr (STENCIL) {
                    const T uw = (e == 0) ? west0 : uc[e - 1];
                    const T ue = (e == E - 1) ? eastL : uc[e + 1];
                    rho[e] = s2 * (rc[e] * (((uw + ue) + (umv[e] + u1[e])) - T(4) * uc[e]));
                } else {
                    rho[e] = A.rho_scale * uc[e];
                }
            }
            // row j is the next row's row j-1: to LDS now, so it is not live in registers
            // across this row's scans
            if constexpr (kUmLds<T, TR>) {
#pragma unroll
                for (int e = 0; e < E; ++e) sh.um[e * TR + t] = uc[e];
            }
        }
        if constexpr (STENCIL) {
            const int ns = sh.src_n;
            if (ns > 0 && live) {
                for (int q = 0; q < ns; ++q) {
                    const int pos = sh.src_pos[q];
                    if ((pos >> 16) == j - j0) {
                        const int i = (pos & 0xffff) - i0;
                        const T add = sh.src_add[q];
#pragma unroll
                        for (int e = 0; e < E; ++e)
                            if (e == i) rho[e] += add;
                    }
                }
            } else if (ns < 0 && live) {
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
        }

        T wout[E];
        xline_row<T, TR>(rho, rc, qc, L, act, lane, wv, j & 1, sh.totf, sh.totb, [&]() {
            if constexpr (kUmLds<T, TR>) load_rq(live ? j + 1 : -1, rn, qn);
        }, wout);
        if constexpr (VEC) bstore8<T>(buf(A.w + (size_t)(live ? j : 0) * nx, live ? row_bytes : 0), voff, wout);
        else if (live && act) gstore8<T>(A.w + (size_t)j * nx, i0, nx, wout);

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

    };

    for (int it = 0; it < RS; ++it) {
        row(it, ua, ub, uc0, ud, ra, rb, qa, qb);
        qa = qb;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if constexpr (!kUmLds<T, TR>) ua[e] = ub[e];
            ub[e] = uc0[e]; uc0[e] = ud[e]; ra[e] = rb[e];
        }
    }
}

// Rows 16-byte aligned with a multiple of 8 values take the 16-byte accesses;
// the choice is uniform over the launch.
template <typename T, int TR, bool FUSE, bool STENCIL = true>
__device__ __forceinline__ void xsweep_strip(const XArgs<T>& A, const int strip, const int t,
                                             XShared<T, TR, FUSE>& sh)
{
    if (A.vec) xsweep_strip_impl<T, TR, FUSE, STENCIL, true>(A, strip, t, sh);
    else xsweep_strip_impl<T, TR, FUSE, STENCIL, false>(A, strip, t, sh);
}

// Receiver values of the level a step launch reads: that level is the previous
// step's result and stays unchanged during this step, so the first workgroup of
// the step's first launch records it (out[k] = u[idx[k]]; an offset outside
// [0, npts) records NaN), and the previous step needs no launch of its own.
template <typename T>
__device__ __forceinline__ void rec_tap(const T* u, const int* idx, T* out, int n, long long npts)
{
    if (n > 0 && blockIdx.x == 0 && blockIdx.y == 0)
        for (int k = threadIdx.x; k < n; k += blockDim.x) {
            const int id = idx[k];
            out[k] = (id >= 0 && id < npts) ? u[id] : T(NAN);
        }
}

// With A.xcd set, the workgroups of one XCD (blockIdx mod 8) take a contiguous band
// of strips, so the rows a strip reads above and below itself, which its
// neighbouring strips read too, come through the same L2 (it pays for strips of a
// few rows, where those rows are a large share of the reads); the grid is a
// multiple of 8 and the workgroups past the last strip exit.
template <typename T, int TR, bool FUSE, bool STENCIL = true>
__global__ void __launch_bounds__(TR >= 256 ? TR : 256) k_xsweep(XArgs<T> A)
{
    rec_tap<T>(A.u, A.rec_idx, A.rec_out, A.nrec, (long long)A.nx * A.ny);
    constexpr int G = (TR >= 256 ? TR : 256) / TR;
    __shared__ XShared<T, TR, FUSE> sh[G];
    const int blk = A.xcd ? (int)((blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3)) : (int)blockIdx.x;
    const int strips = (A.ny + A.rows_per_strip - 1) / A.rows_per_strip;
    if (blk * G >= strips) return;
    const int g = __builtin_amdgcn_readfirstlane(threadIdx.x / TR);   // one group per wavefront or more
    xsweep_strip<T, TR, FUSE, STENCIL>(A, blk * G + g, threadIdx.x - g * TR, sh[g]);
}

// strips in XCD bands: strips of at most this many rows
constexpr int kXcdStripRows = 4;

// x-sweep grid: workgroups for the strips (a multiple of 8 for XCD bands)
inline int xsweep_grid(int ny, int rows_per_strip, int groups_per_wg)
{
    const int strips = (ny + rows_per_strip - 1) / rows_per_strip;
    const int wgs = (strips + groups_per_wg - 1) / groups_per_wg;
    return rows_per_strip <= kXcdStripRows ? (wgs + 7) / 8 * 8 : wgs;
}

}  // namespace adw
