// line_solver.hpp -- exact partition (sub-structuring) solver for one
// tridiagonal line system shared by a group of threads, for gfx950.
//
// The paper solves each line system of the ADI sub-steps (Sec. 2, eqs.
// (fr1)-(fr2)) by cyclic reduction (Sec. 3.1).  Here a line of n unknowns is
// cut into contiguous segments, one per thread; every segment is eliminated
// locally in registers (Gaussian elimination without pivoting), which leaves
// one interface unknown per segment (its last node).  The interface unknowns
// satisfy a tridiagonal reduced system that is solved by parallel cyclic
// reduction in LDS; each thread then back-substitutes its interior.  In exact
// arithmetic this is the same solution as Thomas or cyclic reduction.
//
// Segment s covers nodes [lo_s, lo_s + L_s), its interface unknown is
// X_s = x[lo_s + L_s - 1], its interior the first L_s - 1 nodes.  With X_{s-1}
// and X_s treated as known, the interior solution is
//     x = P + X_{s-1} Lv + X_s Rv,
// where P solves the interior system with the line's right-hand side, Lv with
// -a[lo] e_first and Rv with -c[last interior] e_last.  Substituting the
// first interior value of segment s+1 and the last interior value of segment
// s into the equation of node lo_s + L_s - 1 gives
//     A_s X_{s-1} + B_s X_s + C_s X_{s+1} = D_s
//     A_s = aI Ll_s,  B_s = bI + aI Rl_s + cI Lf_{s+1},  C_s = cI Rf_{s+1},
//     D_s = dI - aI Pl_s - cI Pf_{s+1},
// (f = first interior value, l = last interior value, aI/bI/cI/dI = the
// interface row).  A one-node segment has no interior: its "first interior
// value" is X_s itself (Pf, Lf, Rf) = (0, 0, 1) and its "last interior
// value" is X_{s-1}: (Pl, Ll, Rl) = (0, 1, 0).
#pragma once
#include <hip/hip_runtime.h>

namespace adw {

// Line-operator coefficients of I - beta K L at a node with r = beta kappa / h^2.
template <typename T, int S>
struct CoefR {
    const T (&r)[S];
    __device__ __forceinline__ void get(int k, T& a, T& b, T& c) const {
        a = -r[k];
        b = T(1) + T(2) * r[k];
        c = -r[k];
    }
};

// General coefficients held in registers.
template <typename T, int S>
struct CoefABC {
    const T (&a)[S];
    const T (&b)[S];
    const T (&c)[S];
    __device__ __forceinline__ void get(int k, T& aa, T& bb, T& cc) const {
        aa = a[k];
        bb = b[k];
        cc = c[k];
    }
};

// LDS slots needed per line by partition_solve: 7 * TR values of type T.
template <int TR>
constexpr int partition_lds_slots() { return 7 * TR; }

// Solve one line shared by TR threads.
//   d[S]   in: right-hand side of this thread's segment; out: solution
//   cf     coefficient provider for the segment's nodes (local index k)
//   L      nodes in this thread's segment (0 = thread holds no node)
//   t      segment index of this thread in the line, 0..TR-1
//   nact   number of segments with L > 0 (they are segments 0..nact-1)
//   lds    LDS base of this line; slot of segment q for array v is
//          lds[(v * TR + q) * stride]
//   stride LDS stride between consecutive segments (1 when the line's threads
//          are consecutive lanes; the number of interleaved lines otherwise)
// Every thread of the workgroup must call this the same number of times
// (it contains __syncthreads()).
template <typename T, int S, int TR, class Coef>
__device__ __forceinline__ void partition_solve(T (&d)[S], const Coef& cf, const int L,
                                                const int t, const int nact,
                                                T* __restrict__ lds, const int stride)
{
    T cp[S];   // modified super-diagonal of the interior elimination
    T dl[S];   // response of the interior to the left interface value
    T Pf = T(0), Lf = T(0), Rf = T(1);       // defaults: one-node segment
    T Pl = T(0), Ll = T(1), Rl = T(0);
    T aI = T(0), bI = T(1), cI = T(0), dI = T(0);

#pragma unroll
    for (int k = 0; k < S; ++k) { cp[k] = T(0); dl[k] = T(0); }

    if (L >= 2) {
        // forward elimination over the interior nodes 0..L-2
        T a, b, c;
        cf.get(0, a, b, c);
        T m = T(1) / b;
        cp[0] = c * m;
        d[0] = d[0] * m;
        dl[0] = -a * m;
#pragma unroll
        for (int k = 1; k < S - 1; ++k) {
            if (k < L - 1) {
                cf.get(k, a, b, c);
                m = T(1) / (b - a * cp[k - 1]);
                cp[k] = c * m;
                d[k] = (d[k] - a * d[k - 1]) * m;
                dl[k] = (-a * dl[k - 1]) * m;
            }
        }
        // last interior values and first interior values (back substitution
        // of the three right-hand sides P, Lv, Rv with zero beyond the interior)
        T yP = T(0), yL = T(0), yR = T(1);
#pragma unroll
        for (int k = S - 2; k >= 0; --k) {
            if (k <= L - 2) {
                if (k == L - 2) { Pl = d[k]; Ll = dl[k]; Rl = -cp[k]; }
                yP = d[k] - cp[k] * yP;
                yL = dl[k] - cp[k] * yL;
                yR = -cp[k] * yR;
            }
        }
        Pf = yP; Lf = yL; Rf = yR;
    }
    if (L >= 1) {
#pragma unroll
        for (int k = 0; k < S; ++k)
            if (k == L - 1) { cf.get(k, aI, bI, cI); dI = d[k]; }
    }

    T* bufA = lds;                    // PCR ping buffer: 3 * TR
    T* bufB = lds + 3 * TR * stride;  // PCR pong buffer, first used for the first-value exchange
    T* xsb  = lds + 6 * TR * stride;  // interface solution exchange: TR

    // exchange first interior values with the previous segment
    if (L >= 1) {
        bufB[(0 * TR + t) * stride] = Pf;
        bufB[(1 * TR + t) * stride] = Lf;
        bufB[(2 * TR + t) * stride] = Rf;
    }
    __syncthreads();
    T nPf = T(0), nLf = T(0), nRf = T(0);
    if (t + 1 < nact) {
        nPf = bufB[(0 * TR + t + 1) * stride];
        nLf = bufB[(1 * TR + t + 1) * stride];
        nRf = bufB[(2 * TR + t + 1) * stride];
    }

    // reduced equation of this segment, normalised to a unit diagonal
    T ra = T(0), rc = T(0), rd = T(0);
    if (L >= 1) {
        T A = (t == 0) ? T(0) : aI * Ll;
        T B = bI + aI * Rl + cI * nLf;
        T C = cI * nRf;
        T D = dI - aI * Pl - cI * nPf;
        T inv = T(1) / B;
        ra = A * inv;
        rc = C * inv;
        rd = D * inv;
    }

    // parallel cyclic reduction over the TR interface unknowns
    T* cur = bufA;
    T* oth = bufB;
#pragma unroll
    for (int s = 1; s < TR; s <<= 1) {
        cur[(0 * TR + t) * stride] = ra;
        cur[(1 * TR + t) * stride] = rc;
        cur[(2 * TR + t) * stride] = rd;
        __syncthreads();
        T am = T(0), cm = T(0), dm = T(0), ap = T(0), cpp = T(0), dp = T(0);
        if (t - s >= 0) {
            am = cur[(0 * TR + t - s) * stride];
            cm = cur[(1 * TR + t - s) * stride];
            dm = cur[(2 * TR + t - s) * stride];
        }
        if (t + s < TR) {
            ap = cur[(0 * TR + t + s) * stride];
            cpp = cur[(1 * TR + t + s) * stride];
            dp = cur[(2 * TR + t + s) * stride];
        }
        T bn = T(1) - ra * cm - rc * ap;
        T inv = T(1) / bn;
        T na = -(ra * am) * inv;
        T nc = -(rc * cpp) * inv;
        T nd = (rd - ra * dm - rc * dp) * inv;
        ra = na; rc = nc; rd = nd;
        T* tmp = cur; cur = oth; oth = tmp;
    }
    const T X = rd;

    xsb[t * stride] = X;
    __syncthreads();
    const T Xp = (t > 0) ? xsb[(t - 1) * stride] : T(0);

    // interior back substitution with both interface values known
    if (L >= 2) {
        T x = X;
#pragma unroll
        for (int k = S - 2; k >= 0; --k) {
            if (k <= L - 2) {
                x = (d[k] + Xp * dl[k]) - cp[k] * x;
                d[k] = x;
            }
        }
    }
    if (L >= 1) {
#pragma unroll
        for (int k = 0; k < S; ++k)
            if (k == L - 1) d[k] = X;
    }
}

}  // namespace adw
