// Matrix-free PDHG for the unified Charnes-Cooper LP (Sec. 2.8, Supp. 6.1),
// for one instance or a batch of independent instances advanced in lockstep.
//
// Saddle problem  min_{x in X} max_{lambda >= 0} c^T x + lambda^T (G x - h)
// with x = (y, u, v), D = K P^T y and the rows (band: D - u_bar, gel: D - v_bar U,
// gel: L - D).  One Chambolle-Pock step t = T(z) from z = (y, u, v, lambda):
//
//   q   = P K z_lambda,  z_lambda = lambda_up[band | gel] - lambda_lo[gel]  (Eq. 51)
//   t.y = act ? max(0, y - tau_j q) : 0                                    (Eq. 50)
//   t.u = max(0, u - tau_u (w1 - sum lambda1)),  t.v likewise              (Eq. 48-49)
//   D_t = K P^T t.y,  Dbar = 2 D_t - D(y),  ubar = 2 t.u - u,  vbar = 2 t.v - v
//   t.lambda_up = max(0, lambda_up + s_i (Dbar - ubar | vbar U))           band | gel
//   t.lambda_lo = max(0, lambda_lo + s_i (L - Dbar))                       gel
//
// and the next iterate z+ = w ((1 + rho) t - rho z) + (1 - w) z0 (D carried along
// by linearity):
//   plain mode:     w = 1, rho = 0 (z+ = t), scalar tau = sigma = 0.9 / ||G||
//                   from an FP64 power iteration;
//   restarted mode: reflected Halpern, rho = 1, w = (k+1)/(k+2) with k counted
//                   from the last restart and z0 the restart point; diagonal
//                   Pock-Chambolle steps T_j = 1/colsum_j |G|, S_i = 1/rowsum_i |G|
//                   with a primal weight omega (tau = eta T / omega, sigma =
//                   eta omega S).  Every check_every iterations the PDHG output
//                   t is checked: relative KKT termination, Farkas tests of
//                   lambda(t) - lambda(z) and of lambda(t) - lambda(t at the
//                   previous check), restart rules (sufficient 0.2, necessary
//                   0.8, artificial 0.36) on the l2 merit of the relative KKT
//                   residuals; a restart moves z and z0 to t and updates omega
//                   from the movement since the previous restart.
//
// Batching.  Every instance's arrays are packed into shared workspace fields
// (instance i at element offsets soff_i / voff_i).  Streaming kernels run over
// segment tables (one workgroup = one chunk of one instance), so one launch
// serves all unfinished instances; reductions leave per-workgroup FP64 partials
// that are summed per instance in a fixed order (deterministic).  Single-slice
// instances without blur share one launch per operator (work-item kernels);
// other instances run their plan's operators one after another.  Checks,
// restarts and terminations are decided per instance; a finished instance
// leaves the tables and keeps its returned point untouched.
//
// All iteration-varying scalars live in per-instance device blocks, so an
// iteration is a fixed sequence of launches with fixed arguments; a block of
// iterations can be captured once in a HIP graph and replayed.
#include <algorithm>
#include <chrono>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <vector>

#include "sipo_internal.hpp"

namespace sipo {

constexpr int kNS = 8;                 // sums carried per reduction
constexpr int kThreads = 256;
constexpr long long kChunk = 4096;     // elements per workgroup in segmented launches

// Device scalar block (FP64) of one instance.
struct DevScal {
    double u, v;              // z.u, z.v (Halpern iterate)
    double ut, vt;            // t.u, t.v of the iteration about to run
    double ut_done, vt_done;  // t.u, t.v of the iteration just completed
    double u0, v0;            // anchor scalars
    double ubar, vbar;        // extrapolated scalars for the dual step
    double tau_fac, sig_fac;  // array step factors (eta/omega, eta*omega) or the plain tau, sigma
    double tau_u, tau_v;      // scalar primal steps
    double w, rho;            // Halpern weight of the iteration about to run, reflection
    double k_in;              // iterations since the last restart
    double halpern;           // 1 = restarted mode (w = (k+1)/(k+2)), 0 = plain (w = 1)
    double sum_l1, sum_Ul2;   // sums of the current lambda
    double init_l1, init_Ul2; // lambda sums handed to k_scalars_init
};
static_assert(offsetof(DevScal, rho) == offsetof(DevScal, w) + sizeof(double), "the fused primal step reads (w, rho)");

struct LPConst {
    int u_free, v_free;
    double w1, w2, h;         // weights and band cap
    double lo_s, hi_s;        // scalar bounds when arrays are absent
    double wu, wv;            // column weights of the free scalars in the diagonal steps
};

// Per-instance constants and per-call selectors on the device.
struct InstC {
    LPConst c;
    double eu, ev;            // scalars for KKT / power-iteration evaluations
    double fac;               // per-instance scale factor (power iteration)
    int flag;                 // selects instances for subset operations
    int sel;                  // certificate pair: 0 = (t, pre-step), 1 = (t, snapshot)
};

// One workgroup's share of a segmented launch: instance and packed element range.
struct Seg {
    int inst, pad;
    long long b, e;
};

// -------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

__device__ __forceinline__ void block_sums(double (&v)[kNS], double *partials) {
    __shared__ double red[kThreads / 64][kNS];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kNS; ++k) {
        const double s = wave_sum(v[k]);
        if (lane == 0) red[w][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < kNS) {
        double s = 0.0;
        for (int i = 0; i < kThreads / 64; ++i) s += red[i][threadIdx.x];
        partials[blockIdx.x * kNS + threadIdx.x] = s;
    }
}

// block_sums for kernels whose consumers read columns 0 and 1 only (the others are left as they are)
__device__ __forceinline__ void block_sums2(double a, double b, double *partials) {
    __shared__ double red2[kThreads / 64][2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const double sa = wave_sum(a), sb = wave_sum(b);
    if (lane == 0) { red2[w][0] = sa; red2[w][1] = sb; }
    __syncthreads();
    if (threadIdx.x < 2) {
        double s = 0.0;
        for (int i = 0; i < kThreads / 64; ++i) s += red2[i][threadIdx.x];
        partials[blockIdx.x * kNS + threadIdx.x] = s;
    }
}

// Total of column k over partials[first .. first + count), by one block: strided
// per-thread sums, then a fixed tree, so the result does not depend on timing.
template <bool MAX>
__device__ double block_total(const double *__restrict__ partials, int first, int count, int k, double *sh) {
    double a = 0.0;
    for (int b = threadIdx.x; b < count; b += kThreads) {
        const double v = partials[(size_t)(first + b) * kNS + k];
        a = MAX ? fmax(a, v) : a + v;
    }
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] = MAX ? fmax(sh[threadIdx.x], sh[threadIdx.x + o])
                                                       : sh[threadIdx.x] + sh[threadIdx.x + o];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Columns 0 and 1 of partials[first .. first + count) at once, by one block: each thread adds its rows
// b = t, t + kThreads, ... in that order (one 16-byte load per row, four rows in flight), then one fixed
// tree; per column the additions are the ones block_total<false> makes, in the same order.
__device__ double2 block_total01(const double *__restrict__ partials, int first, int count, double2 *sh) {
    double a0 = 0.0, a1 = 0.0;
    for (int b0 = threadIdx.x; b0 < count; b0 += 4 * kThreads) {
        double2 v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            v[q] = *(const double2 *)(partials + (size_t)(first + min(b0 + q * kThreads, count - 1)) * kNS);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (b0 + q * kThreads < count) {
                a0 += v[q].x;
                a1 += v[q].y;
            }
    }
    sh[threadIdx.x] = make_double2(a0, a1);
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const double2 x = sh[threadIdx.x], y = sh[threadIdx.x + o];
            sh[threadIdx.x] = make_double2(x.x + y.x, x.y + y.y);
        }
        __syncthreads();
    }
    const double2 r = sh[0];
    __syncthreads();
    return r;
}

// out[i][k] for the instances i = list[blockIdx.x]: totals of their workgroups' partials.
template <bool MAX>
__global__ void __launch_bounds__(kThreads) k_finish(const double *__restrict__ partials, const int *__restrict__ first,
                                                      const int *__restrict__ count, const int *__restrict__ list,
                                                      int ns, double *__restrict__ out) {
    __shared__ double sh[kThreads];
    const int i = list[blockIdx.x];
    for (int k = 0; k < ns; ++k) {
        const double r = block_total<MAX>(partials, first[i], count[i], k, sh);
        if (threadIdx.x == 0) out[(size_t)i * kNS + k] = r;
    }
}

#define SEG_LOOP(i) \
    const Seg sg_ = segs[blockIdx.x]; \
    for (long long i = sg_.b + threadIdx.x; i < sg_.e; i += kThreads)

template <typename T>
__device__ __forceinline__ T ld_or(const T *p, long long i, double s) { return p ? p[i] : (T)s; }

// ------------------------------------------------------------ setup kernels
// y <- act ? max(y, 0) : 0  (warm start projected onto X)
template <typename T>
__global__ void k_project_y(T *y, const uint8_t *act, const Seg *segs) {
    SEG_LOOP(i) y[i] = act[i] ? (y[i] > (T)0 ? y[i] : (T)0) : (T)0;
}

// lambda projected onto its regions and >= 0; z = lambda_up - lambda_lo; [0] sum_band lambda1, [1] sum_gel U lambda2.
template <typename T>
__global__ void k_lambda_z(T *lu, T *ll, T *z, const uint8_t *lab, const T *hi, const InstC *insts, const Seg *segs,
                           int use_flag, double *partials) {
    double acc[kNS] = {0, 0, 0, 0, 0, 0, 0, 0};
    const InstC &ic = insts[segs[blockIdx.x].inst];
    if (!use_flag || ic.flag) {
        SEG_LOOP(i) {
            const uint8_t L = lab[i];
            T a = L ? (lu[i] > (T)0 ? lu[i] : (T)0) : (T)0;
            T b = (L == 2) ? (ll[i] > (T)0 ? ll[i] : (T)0) : (T)0;
            lu[i] = a;
            ll[i] = b;
            z[i] = a - b;
            if (L == 1) acc[0] += (double)a;
            if (L == 2) acc[1] += (double)ld_or(hi, i, ic.c.hi_s) * (double)a;
        }
    }
    block_sums(acc, partials);
}

// w = 1 on band, 2 on gel (absolute column weights of G)
template <typename T>
__global__ void k_colweight(T *w, const uint8_t *lab, const Seg *segs) {
    SEG_LOOP(i) w[i] = lab[i] == 1 ? (T)1 : (lab[i] == 2 ? (T)2 : (T)0);
}

template <typename T>
__global__ void k_act_to_float(T *a, const uint8_t *act, const Seg *segs) {
    SEG_LOOP(i) a[i] = act[i] ? (T)1 : (T)0;
}

// T_j = act & colsum > 0 ? 1 / colsum : 0
template <typename T>
__global__ void k_inv_colsum(T *t, const uint8_t *act, const Seg *segs) {
    SEG_LOOP(i) t[i] = (act[i] && t[i] > (T)0) ? (T)1 / t[i] : (T)0;
}

// S_up = 1/(R + [band, u free] w_u + [gel, v free] w_v U), S_lo = [gel] 1/R (weighted
// Pock-Chambolle steps: the free scalars' columns carry weights w_u, w_v, their steps are
// w_u / |band| and w_v / sum_gel U, and the bound on the preconditioned operator holds for any
// positive weights);
// [0] |band|, [1] sum_gel U, [2] ||h||^2, [3] |gel|, [4] sum_band R, [5] sum_gel R U
template <typename T>
__global__ void k_row_scaling(const T *R, T *s_up, T *s_lo, const uint8_t *lab, const T *lo, const T *hi,
                              const InstC *insts, const Seg *segs, double *partials) {
    double acc[kNS] = {0, 0, 0, 0, 0, 0, 0, 0};
    const LPConst c = insts[segs[blockIdx.x].inst].c;
    SEG_LOOP(i) {
        const uint8_t L = lab[i];
        const T r = R[i];
        T su = 0, sl = 0;
        if (L == 1) {
            const T rs = r + (c.u_free ? (T)c.wu : (T)0);
            su = rs > (T)0 ? (T)1 / rs : (T)0;
            acc[0] += 1.0;
            acc[4] += (double)r;
            if (!c.u_free) acc[2] += c.h * c.h;
        } else if (L == 2) {
            const double U = (double)ld_or(hi, i, c.hi_s), Lo = (double)ld_or(lo, i, c.lo_s);
            const T rs = r + (c.v_free ? (T)(c.wv * U) : (T)0);
            su = rs > (T)0 ? (T)1 / rs : (T)0;
            sl = r > (T)0 ? (T)1 / r : (T)0;
            acc[1] += U;
            acc[2] += Lo * Lo + (c.v_free ? 0.0 : U * U);
            acc[3] += 1.0;
            acc[5] += (double)r * U;
        }
        s_up[i] = su;
        s_lo[i] = sl;
    }
    block_sums(acc, partials);
}

// --------------------------------------------------------- iteration kernels
// The iteration kernels give each thread kPer consecutive elements of its segment, one 16-byte
// test of the mask bytes for all of them, and four-element vector accesses.  Segments start on
// multiples of 64 elements and every packed array has the same padding after each instance, so the
// kPer elements starting at an index below the segment's end are always inside the allocation:
// elements past the end (the packing gap) are loaded but never stored.
constexpr int kPer = (int)(kChunk / kThreads);
static_assert(kPer == 16, "one 16-byte mask word per thread");

template <typename T> struct Q4 { T v[4]; };

template <typename T>
__device__ __forceinline__ Q4<T> ld4(const T *p) {
    Q4<T> r;
    if constexpr (sizeof(T) == 4) {
        const float4 a = *(const float4 *)p;
        r.v[0] = a.x; r.v[1] = a.y; r.v[2] = a.z; r.v[3] = a.w;
    } else {
        const double2 a = ((const double2 *)p)[0], b = ((const double2 *)p)[1];
        r.v[0] = a.x; r.v[1] = a.y; r.v[2] = b.x; r.v[3] = b.y;
    }
    return r;
}

template <typename T>
__device__ __forceinline__ void st4(T *p, const Q4<T> &r) {
    if constexpr (sizeof(T) == 4) {
        *(float4 *)p = make_float4(r.v[0], r.v[1], r.v[2], r.v[3]);
    } else {
        ((double2 *)p)[0] = make_double2(r.v[0], r.v[1]);
        ((double2 *)p)[1] = make_double2(r.v[2], r.v[3]);
    }
}

// all four bytes of a mask word nonzero
__device__ __forceinline__ bool all_bytes(uint32_t w) { return ((w - 0x01010101u) & ~w & 0x80808080u) == 0; }
__device__ __forceinline__ uint32_t byte_of(uint32_t w, int k) { return (w >> (8 * k)) & 0xFFu; }

// live[s] = 1 when some mask byte of segment s is nonzero (one workgroup per segment)
__global__ void __launch_bounds__(kThreads) k_seg_live(const uint8_t *__restrict__ m, const Seg *__restrict__ segs,
                                                       uint8_t *__restrict__ live) {
    const Seg sg = segs[blockIdx.x];
    const long long i0 = sg.b + (long long)kPer * threadIdx.x;
    bool any = false;
    if (i0 < sg.e) {
        const uint4 v = *(const uint4 *)(m + i0);
        const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
        const long long n = sg.e - i0;   // bytes of the segment (the rest is packing gap)
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
            for (int k = 0; k < 4; ++k) any = any || (4 * g + k < n && byte_of(w4[g], k) != 0);
    }
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) live[blockIdx.x] = any ? 1 : 0;
}

// Optional fields known at compile time.  A kernel variant either loads a field or uses its
// constant, so every load of the variant is unconditional and the compiler issues them back to back
// and waits once; a pointer test per field had put a branch around each load and a full memory wait
// after some of them.  HAL = Halpern anchors and row scalings present (restarted mode); BND =
// per-voxel bounds present.
template <bool HAS, typename T>
__device__ __forceinline__ Q4<T> ld4_if(const T *p, long long i, double s) {
    if constexpr (HAS) {
        return ld4(p + i);
    } else {
        Q4<T> r;
        r.v[0] = r.v[1] = r.v[2] = r.v[3] = (T)s;
        return r;
    }
}

// t.y = act ? max(0, y - tau q) : 0 with tau = tau_fac T_j (or tau_fac); y <- w ((1+rho) t.y - rho y) + (1-w) y0.
// A masked ray keeps y = t.y = anchor = 0 (all three start at zero there), so it is not stored.
template <typename T, bool HAL>
__global__ void __launch_bounds__(kThreads) k_primal(T *__restrict__ y, T *__restrict__ yt, const T *__restrict__ q,
                                                     const T *__restrict__ Tj, const uint8_t *__restrict__ act,
                                                     const T *__restrict__ y0, const DevScal *__restrict__ scal,
                                                     const Seg *__restrict__ segs) {
    const Seg sg = segs[blockIdx.x];
    const long long i0 = sg.b + (long long)kPer * threadIdx.x;
    if (i0 >= sg.e) return;
    const uint4 m = *(const uint4 *)(act + i0);
    if (!(m.x | m.y | m.z | m.w)) return;
    const DevScal &sc = scal[sg.inst];
    const T tf = (T)sc.tau_fac;
    const T w = (T)sc.w, rho = (T)sc.rho;
    const uint32_t mw[4] = {m.x, m.y, m.z, m.w};
    Q4<T> yo[4], qq[4], tj[4], a0[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        yo[g] = ld4(y + i0 + 4 * g);
        qq[g] = ld4(q + i0 + 4 * g);
        tj[g] = ld4_if<HAL>(Tj, i0 + 4 * g, 1.0);
        a0[g] = ld4_if<HAL>(y0, i0 + 4 * g, 0.0);
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        Q4<T> t, yn;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            T v = yo[g].v[k] - tf * tj[g].v[k] * qq[g].v[k];
            v = v > (T)0 ? v : (T)0;
            t.v[k] = v;
            yn.v[k] = HAL ? w * (((T)1 + rho) * v - rho * yo[g].v[k]) + ((T)1 - w) * a0[g].v[k] : v;
        }
        const long long ib = i0 + 4 * g;
        if (all_bytes(mw[g]) && ib + 4 <= sg.e) {
            st4(yt + ib, t);
            st4(y + ib, yn);
        } else if (mw[g]) {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (ib + k < sg.e && byte_of(mw[g], k)) { yt[ib + k] = t.v[k]; y[ib + k] = yn.v[k]; }
        }
    }
}

// Dual step on voxels from D_t (= K P^T t.y) and D (= K P^T z.y); Halpern update of lambda and D;
// z_lambda for the next step; on check iterations t.lambda and the pre-step lambda are kept.
// [0] sum_band lambda1, [1] sum_gel U lambda2 of the new lambda.  LAB (labelled only): the dose of
// unlabelled voxels is not kept (nothing reads it during the solve), so a thread whose voxels are
// all unlabelled does nothing.  The voxels of a thread are handled in two halves of eight, each
// with all of its loads issued before its arithmetic.
// HAL and BND: see ld4_if.
template <typename T, bool HAL, bool BND, bool LAB>
__global__ void __launch_bounds__(kThreads) k_dual(
    const T *__restrict__ Dt, T *__restrict__ D, const T *__restrict__ D0, T *__restrict__ lu, T *__restrict__ ll,
    const T *__restrict__ lu0, const T *__restrict__ ll0, T *__restrict__ z, const uint8_t *__restrict__ lab,
    const T *__restrict__ lo, const T *__restrict__ hi, const T *__restrict__ s_up, const T *__restrict__ s_lo,
    T *__restrict__ lut, T *__restrict__ llt, T *__restrict__ luo, T *__restrict__ llo,
    const DevScal *__restrict__ scal, const InstC *__restrict__ insts, const Seg *__restrict__ segs, double *partials) {
    const Seg sg = segs[blockIdx.x];
    const DevScal &sc = scal[sg.inst];
    const LPConst c = insts[sg.inst].c;
    const T sf = (T)sc.sig_fac;
    const T ub = (T)(c.u_free ? sc.ubar : c.h);
    const T vb = (T)(c.v_free ? sc.vbar : 1.0);
    const T w = (T)sc.w, rho = (T)sc.rho, w1 = (T)1 - w, rp = (T)1 + rho;
    double acc[2] = {0, 0};   // the consumers (k_scalars) read these two columns only
    const long long i0 = sg.b + (long long)kPer * threadIdx.x;
    uint4 l16 = make_uint4(0u, 0u, 0u, 0u);
    if (i0 < sg.e) l16 = *(const uint4 *)(lab + i0);
    const uint32_t lw[4] = {l16.x, l16.y, l16.z, l16.w};
    const bool any_label = (l16.x | l16.y | l16.z | l16.w) != 0;
    if (i0 < sg.e && (!LAB || any_label)) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            Q4<T> dt[2], dz[2], d0[2], a_old[2], a_0[2], su[2], U[2], b_old[2], b_0[2], sl[2], Lo[2];
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                const long long ib = i0 + 4 * (2 * h + g);
                dt[g] = ld4(Dt + ib);
                dz[g] = ld4(D + ib);
                d0[g] = ld4_if<HAL>(D0, ib, 0.0);
                a_old[g] = ld4(lu + ib);
                a_0[g] = ld4_if<HAL>(lu0, ib, 0.0);
                su[g] = ld4_if<HAL>(s_up, ib, 1.0);
                U[g] = ld4_if<BND>(hi, ib, c.hi_s);
                b_old[g] = ld4(ll + ib);
                b_0[g] = ld4_if<HAL>(ll0, ib, 0.0);
                sl[g] = ld4_if<HAL>(s_lo, ib, 1.0);
                Lo[g] = ld4_if<BND>(lo, ib, c.lo_s);
            }
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                const uint32_t L4 = lw[2 * h + g];
                const long long ib = i0 + 4 * (2 * h + g);
                Q4<T> dn, an, at, bn, bt, zz;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t L = byte_of(L4, k);
                    const T t = dt[g].v[k], d = dz[g].v[k];
                    dn.v[k] = HAL ? w * (rp * t - rho * d) + w1 * d0[g].v[k] : t;
                    const T Db = (T)2 * t - d;
                    T a = a_old[g].v[k] + sf * su[g].v[k] * (Db - (L == 1 ? ub : vb * U[g].v[k]));
                    a = a > (T)0 ? a : (T)0;
                    at.v[k] = a;
                    an.v[k] = HAL ? w * (rp * a - rho * a_old[g].v[k]) + w1 * a_0[g].v[k] : a;
                    T b = b_old[g].v[k] + sf * sl[g].v[k] * (Lo[g].v[k] - Db);
                    b = b > (T)0 ? b : (T)0;
                    bt.v[k] = b;
                    bn.v[k] = HAL ? w * (rp * b - rho * b_old[g].v[k]) + w1 * b_0[g].v[k] : b;
                    zz.v[k] = L == 2 ? an.v[k] - bn.v[k] : an.v[k];
                    if (ib + k < sg.e) {
                        if (L == 1) acc[0] += (double)an.v[k];
                        if (L == 2) acc[1] += (double)U[g].v[k] * (double)an.v[k];
                    }
                }
                // D, lambda and z are stored as whole 16-byte words with no branch, so the compiler can
                // count the stores in its waits: an element that is not updated (not labelled, or past
                // the segment end, in the packing gap that nothing reads) gets back the value loaded
                // for it, or 0 for z (z, lambda_up and lambda_lo are zero off their labels).  The dose
                // of an unlabelled voxel is stored too: it is either kept or not read.
                Q4<T> dS, luS, zS, llS;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const bool in = ib + k < sg.e;
                    const uint32_t L = byte_of(L4, k);
                    dS.v[k] = in ? dn.v[k] : dz[g].v[k];
                    luS.v[k] = (in && L) ? an.v[k] : a_old[g].v[k];
                    zS.v[k] = (in && L) ? zz.v[k] : (T)0;
                    llS.v[k] = (in && L == 2) ? bn.v[k] : b_old[g].v[k];
                }
                st4(D + ib, dS);
                if (LAB || any_label) {   // LAB: the thread holds a label, no test needed
                    st4(lu + ib, luS);
                    st4(z + ib, zS);
                    st4(ll + ib, llS);
                }
                // check iterations only: the restart copies take these fields over whole segments, so
                // they are written on labelled voxels alone
                if (lut) {
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (ib + k < sg.e && byte_of(L4, k)) {
                            lut[ib + k] = at.v[k];
                            luo[ib + k] = a_old[g].v[k];
                            if (byte_of(L4, k) == 2) {
                                llt[ib + k] = bt.v[k];
                                llo[ib + k] = b_old[g].v[k];
                            }
                        }
                }
            }
        }
    }
    block_sums2(acc[0], acc[1], partials);
}

template <typename T, bool LAB>
static auto dual_kernel_l(bool hal, bool bnd) -> decltype(&k_dual<T, true, true, LAB>) {
    if (hal) return bnd ? &k_dual<T, true, true, LAB> : &k_dual<T, true, false, LAB>;
    return bnd ? &k_dual<T, false, true, LAB> : &k_dual<T, false, false, LAB>;
}

template <typename T>
static auto dual_kernel(bool hal, bool bnd, bool lab) -> decltype(&k_dual<T, true, true, true>) {
    return lab ? dual_kernel_l<T, true>(hal, bnd) : dual_kernel_l<T, false>(hal, bnd);
}

// Next scalar primal step from the current z and the lambda sums.
__device__ __forceinline__ void roll_next(DevScal *sc, const LPConst &c) {
    sc->ut = c.u_free ? fmax(0.0, sc->u - sc->tau_u * (c.w1 - sc->sum_l1)) : c.h;
    sc->vt = c.v_free ? fmax(0.0, sc->v - sc->tau_v * (c.w2 - sc->sum_Ul2)) : 1.0;
    sc->ubar = 2.0 * sc->ut - sc->u;
    sc->vbar = 2.0 * sc->vt - sc->v;
}

// One block per listed instance: finish its lambda sums, Halpern update of (u, v), next step.
__global__ void __launch_bounds__(kThreads) k_scalars(const double *__restrict__ partials,
                                                       const int *__restrict__ first, const int *__restrict__ count,
                                                       const int *__restrict__ list, DevScal *scal,
                                                       const InstC *__restrict__ insts) {
    __shared__ double2 sh[kThreads];
    const int i = list[blockIdx.x];
    const double2 s01 = block_total01(partials, first[i], count[i], sh);
    const double s0 = s01.x, s1 = s01.y;
    if (threadIdx.x != 0) return;
    DevScal *sc = scal + i;
    const LPConst c = insts[i].c;
    const double w = sc->w, rho = sc->rho;
    sc->ut_done = sc->ut;
    sc->vt_done = sc->vt;
    if (c.u_free) sc->u = w * ((1.0 + rho) * sc->ut - rho * sc->u) + (1.0 - w) * sc->u0;
    else sc->u = c.h;
    if (c.v_free) sc->v = w * ((1.0 + rho) * sc->vt - rho * sc->v) + (1.0 - w) * sc->v0;
    else sc->v = 1.0;
    sc->sum_l1 = s0;
    sc->sum_Ul2 = s1;
    sc->k_in += 1.0;
    sc->w = sc->halpern != 0.0 ? (sc->k_in + 1.0) / (sc->k_in + 2.0) : 1.0;
    roll_next(sc, c);
}

// After a (re)start of the flagged instances: lambda sums from init_*, Halpern weight, first step.
__global__ void k_scalars_init(DevScal *scal, const InstC *insts, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        if (!insts[i].flag) continue;
        DevScal *sc = scal + i;
        sc->sum_l1 = sc->init_l1;
        sc->sum_Ul2 = sc->init_Ul2;
        sc->k_in = 0.0;
        sc->w = sc->halpern != 0.0 ? 0.5 : 1.0;
        roll_next(sc, insts[i].c);
    }
}

// ---------------------------------------------------------------- KKT pieces
// Voxel side at (D, eu, ev, lambda): [0] ||(Gx-h)^+||^2 voxel rows, [1] sum L lambda3,
// [2] sum_band lambda1, [3] sum_gel U lambda2.
template <typename T>
__global__ void k_kkt_vox(const T *D, const T *lu, const T *ll, const uint8_t *lab, const T *lo, const T *hi,
                          const InstC *insts, const Seg *segs, double *partials) {
    double acc[kNS] = {0, 0, 0, 0, 0, 0, 0, 0};
    const InstC &ic = insts[segs[blockIdx.x].inst];
    const LPConst c = ic.c;
    const double u = ic.eu, v = ic.ev;
    SEG_LOOP(i) {
        const uint8_t L = lab[i];
        if (L == 0) continue;
        const double d = (double)D[i];
        if (L == 1) {
            const double r = d - (c.u_free ? u : c.h);
            if (r > 0) acc[0] += r * r;
            acc[2] += (double)lu[i];
        } else {
            const double U = (double)ld_or(hi, i, c.hi_s), Lo = (double)ld_or(lo, i, c.lo_s);
            const double r1 = d - (c.v_free ? v : 1.0) * U, r2 = Lo - d;
            if (r1 > 0) acc[0] += r1 * r1;
            if (r2 > 0) acc[0] += r2 * r2;
            acc[1] += Lo * (double)ll[i];
            acc[3] += U * (double)lu[i];
        }
    }
    block_sums(acc, partials);
}

// Ray side: [0] sum_act min(q,0)^2, [1] sum_act y^-^2 + sum_mask y^2.
template <typename T>
__global__ void k_kkt_ray(const T *q, const T *y, const uint8_t *act, const Seg *segs, double *partials) {
    double acc[kNS] = {0, 0, 0, 0, 0, 0, 0, 0};
    SEG_LOOP(i) {
        const double yi = (double)y[i];
        if (act[i]) {
            const double qi = (double)q[i];
            if (qi < 0) acc[0] += qi * qi;
            if (yi < 0) acc[1] += yi * yi;
        } else {
            acc[1] += yi * yi;
        }
    }
    block_sums(acc, partials);
}

// Farkas candidate d = max(a - b, 0) on the regions of the flagged instances -> z_d (b = NULL: the
// candidate is max(a, 0) itself); [0] sum L d3, [1] sum_band d1, [2] sum_gel U d2, [3] ||d||_1.
template <typename T>
__global__ void k_ray_candidate(const T *alu, const T *all, const T *blu, const T *bll, T *zd, const uint8_t *lab,
                                const T *lo, const T *hi, const InstC *insts, const Seg *segs, double *partials) {
    double acc[kNS] = {0, 0, 0, 0, 0, 0, 0, 0};
    const InstC &ic = insts[segs[blockIdx.x].inst];
    if (ic.flag) {
        const LPConst c = ic.c;
        SEG_LOOP(i) {
            const uint8_t L = lab[i];
            T zz = 0;
            if (L) {
                T a = alu[i] - (blu ? blu[i] : (T)0);
                a = a > (T)0 ? a : (T)0;
                zz = a;
                acc[3] += (double)a;
                if (L == 1) {
                    acc[1] += (double)a;
                } else {
                    T b = all[i] - (bll ? bll[i] : (T)0);
                    b = b > (T)0 ? b : (T)0;
                    zz = a - b;
                    acc[0] += (double)ld_or(lo, i, c.lo_s) * (double)b;
                    acc[2] += (double)ld_or(hi, i, c.hi_s) * (double)a;
                    acc[3] += (double)b;
                }
            }
            zd[i] = zz;
        }
    }
    block_sums(acc, partials);
}

// Certificate output of the flagged instances: max(a - b, 0) on the regions (b = NULL: max(a, 0)).
template <typename T>
__global__ void k_certificate(T *olu, T *oll, const T *alu, const T *all, const T *blu, const T *bll,
                              const uint8_t *lab, const InstC *insts, const Seg *segs) {
    const InstC &ic = insts[segs[blockIdx.x].inst];
    if (!ic.flag) return;
    SEG_LOOP(i) {
        const uint8_t L = lab[i];
        T a = L ? alu[i] - (blu ? blu[i] : (T)0) : (T)0;
        T b = (L == 2) ? all[i] - (bll ? bll[i] : (T)0) : (T)0;
        olu[i] = a > (T)0 ? a : (T)0;
        oll[i] = b > (T)0 ? b : (T)0;
    }
}

// [0] max over act of -q (clipped at 0), [1] max over act of |q|
template <typename T>
__global__ void k_ray_check(const T *q, const uint8_t *act, const Seg *segs, double *partials) {
    __shared__ double m0[kThreads], m1[kThreads];
    double a0 = 0.0, a1 = 0.0;
    SEG_LOOP(i) {
        if (!act[i]) continue;
        const double qi = (double)q[i];
        a0 = fmax(a0, -qi);
        a1 = fmax(a1, fabs(qi));
    }
    m0[threadIdx.x] = a0;
    m1[threadIdx.x] = a1;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            m0[threadIdx.x] = fmax(m0[threadIdx.x], m0[threadIdx.x + o]);
            m1[threadIdx.x] = fmax(m1[threadIdx.x], m1[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[blockIdx.x * kNS + 0] = m0[0];
        partials[blockIdx.x * kNS + 1] = m1[0];
    }
}

// power iteration: the rows of G x with D = K P^T y and the scalars (eu, ev) combined for G^T:
// z = (D - eu) on band, (D - ev U) + D on gel; [0] sum_band (D - eu), [1] sum_gel U (D - ev U)
template <typename T>
__global__ void k_pi_rows(const T *D, T *z, const uint8_t *lab, const T *hi, const InstC *insts, const Seg *segs,
                          double *partials) {
    double acc[kNS] = {0, 0, 0, 0, 0, 0, 0, 0};
    const InstC &ic = insts[segs[blockIdx.x].inst];
    const LPConst c = ic.c;
    SEG_LOOP(i) {
        const uint8_t L = lab[i];
        T zz = 0;
        if (L == 1) {
            const double r = (double)D[i] - (c.u_free ? ic.eu : 0.0);
            zz = (T)r;
            acc[0] += r;
        } else if (L == 2) {
            const double U = (double)ld_or(hi, i, c.hi_s);
            const double r = (double)D[i] - (c.v_free ? ic.ev * U : 0.0);
            zz = (T)(r + (double)D[i]);   // gel-up row minus gel-lo row (-D)
            acc[1] += U * r;
        }
        z[i] = zz;
    }
    block_sums(acc, partials);
}

// y <- act ? q : 0 ; [0] sum y^2
template <typename T>
__global__ void k_pi_mask(T *y, const T *q, const uint8_t *act, const Seg *segs, double *partials) {
    double acc[kNS] = {0, 0, 0, 0, 0, 0, 0, 0};
    SEG_LOOP(i) {
        const T v = act[i] ? q[i] : (T)0;
        y[i] = v;
        acc[0] += (double)v * (double)v;
    }
    block_sums(acc, partials);
}

template <typename T>
__global__ void k_scale(T *a, const InstC *insts, const Seg *segs) {
    const double s = insts[segs[blockIdx.x].inst].fac;
    SEG_LOOP(i) a[i] = (T)((double)a[i] * s);
}

// dst <- src on all listed instances, or only on flagged ones
template <typename T>
__global__ void k_copy(T *dst, const T *src, const InstC *insts, const Seg *segs, int use_flag) {
    if (use_flag && !insts[segs[blockIdx.x].inst].flag) return;
    SEG_LOOP(i) dst[i] = src[i];
}

template <typename T>
__global__ void k_fill(T *dst, long long n, T v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        dst[i] = v;
}

// weighted movement: [0] sum (a-b)^2 / w over w > 0
template <typename T>
__global__ void k_wdist(const T *a, const T *b, const T *w, const Seg *segs, double *partials) {
    double acc[kNS] = {0, 0, 0, 0, 0, 0, 0, 0};
    SEG_LOOP(i) {
        const double wi = (double)w[i];
        if (wi > 0) {
            const double d = (double)a[i] - (double)b[i];
            acc[0] += d * d / wi;
        }
    }
    block_sums(acc, partials);
}

// ================================================================= host side
static size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }
static long long align_elems(long long v) { return (v + 63) & ~63LL; }

// Byte offsets of everything in the caller's workspace.
struct Layout {
    int B = 0;
    std::vector<long long> soff, voff;          // element offsets per instance
    long long NS = 0, NV = 0;                   // packed sizes (elements)
    int max_seg_s = 0, max_seg_v = 0, max_items_bp = 0, max_items_fp = 0, max_items_tr = 0;
    size_t eb = 4;
    bool lohi = false;                          // per-voxel bounds packed (some instance has arrays)
    size_t vol_t_elems = 0;                     // largest 3D instance (the projector's input is per instance)
    std::vector<size_t> pfo, bfo;               // byte offsets of each 3D instance's skip flags
    std::vector<size_t> pso, pco;               // and of its projector step lists and step counts
    size_t ps_bytes = 0, pc_bytes = 0, reach_bytes = 0;
    size_t psteps = 0, pcount = 0, preach = 0;  // their fields; the reach masks of the list builder
    size_t pitems = 0, pqueue = 0;              // the projector's work queue: tiles (offsets pco) and counters
    std::vector<size_t> bno;                    // and of its backprojector's per-column need mask
    size_t bn_bytes = 0, bneed = 0;
    std::vector<size_t> kfo;                    // and of its two blur tile flag arrays (own, reach)
    size_t kf_bytes = 0, kflags = 0;
    size_t pf_bytes = 0, bf_bytes = 0;          // projector / backprojector flag totals
    size_t pflags = 0, bflags = 0;              // their fields
    size_t part_s = 0, part_v = 0;              // elements of the largest 3D instance's sinogram / volume
    size_t ppart = 0, bpart = 0;                // partial sums of the split 3D operators
    // sinogram fields
    size_t y, q, Tj, yt, y0, ylast, act;
    // volume fields
    size_t lu, ll, D, Dt, D0, z, tmp, tmp2, s_up, s_lo, lut, llt, luo, llo, snap_u, snap_l, lu0, ll0, lul, lll, lab,
        lo, hi, vol_t;
    // tables
    size_t segSL = 0, segVL = 0, firstVL = 0, cntVL = 0, live = 0;   // tables of the segments with work
    size_t partials, insts, scal, segS, segV, firstS, cntS, firstV, cntV, list_act, list_tmp, sums, geo, items_bp,
        items_fp, items_tr;
    size_t total = 0;
};

constexpr size_t kNoField = ~(size_t)0;   // "no field": the Farkas candidate is lambda itself

// Largest splits of the 3D projector's march and of the backprojector's views in LP solves.
constexpr int kMaxSplitP = 4, kMaxSplitB = 8;
// slices per blur tile in masked solves: a blur workgroup streams its slices and the PSF halo one by
// one, so the few tiles left on run shortest with short chunks
constexpr int kMaskBlurZc = 4;
constexpr size_t kQueueStride = 256;   // bytes per instance of the projector's work-queue counters
constexpr double kTuneMargin = 0.98;   // a tuning candidate must beat the best so far by 2 %

// The 2D pair's work shapes the batched solver's tuner tries, in preference order (the default first).
static std::vector<Tiles2D> tiles2d_candidates() {
    std::vector<Tiles2D> out;
    for (int shape = 0; shape < 3; ++shape)
        for (int vb : {16, 8, 32}) {
            Tiles2D t;
            t.bx = shape == 0 ? 32 : shape == 1 ? 16 : 64;
            t.by = 256 / t.bx;
            t.vb = vb;
            out.push_back(t);
        }
    for (int fb : {32, 128}) {
        Tiles2D t;
        t.fb = fb;
        out.push_back(t);
    }
    return out;
}

static bool use_batch2d(const sipo_problem *probs, int B) {
    for (int i = 0; i < B; ++i) {
        const sipo_plan p = probs[i].plan;
        if (!(p->nz == 1 && p->p2d_ok && !p->has_psf)) return false;
    }
    return true;
}

static Layout make_layout(const sipo_problem *probs, int B) {
    Layout L;
    L.B = B;
    L.eb = probs[0].plan->elem_bytes();
    L.soff.resize(B);
    L.voff.resize(B);
    L.pfo.assign(B, 0);
    L.bfo.assign(B, 0);
    L.pso.assign(B, 0);
    L.pco.assign(B, 0);
    L.kfo.assign(B, 0);
    L.bno.assign(B, 0);
    const bool b2d = use_batch2d(probs, B);
    for (int i = 0; i < B; ++i) {
        const sipo_plan p = probs[i].plan;
        const long long ns = (long long)p->sino_elems(), nv = (long long)p->vol_elems();
        L.soff[i] = L.NS;
        L.voff[i] = L.NV;
        L.NS += align_elems(ns);
        L.NV += align_elems(nv);
        L.max_seg_s += (int)((ns + kChunk - 1) / kChunk);
        L.max_seg_v += (int)((nv + kChunk - 1) / kChunk);
        if (probs[i].lo || probs[i].hi) L.lohi = true;
        if (p->fast3d()) {
            L.vol_t_elems = std::max(L.vol_t_elems, (size_t)nv);
            L.pfo[i] = L.pf_bytes;
            L.bfo[i] = L.bf_bytes;
            // room for the finest slice counts the solve may switch to (8 and 4 slices per thread)
            L.pf_bytes += align_up(p3d_flag_count(p, 8));
            L.bf_bytes += align_up(bp3d_flag_count(p, 4));
            L.pso[i] = L.ps_bytes;
            L.pco[i] = L.pc_bytes;
            L.ps_bytes += align_up(sizeof(int) * p3d_flag_count(p, 8) * (size_t)p->n);
            L.pc_bytes += align_up(sizeof(int) * p3d_flag_count(p, 8));
            L.reach_bytes = std::max(L.reach_bytes, std::max(p3d_reach_bytes(p, 8), bp3d_need_bytes(p, 4)));
            L.bno[i] = L.bn_bytes;
            L.bn_bytes += align_up(bp3d_need_bytes(p, 4));
            L.kfo[i] = L.kf_bytes;
            L.kf_bytes += 2 * align_up(blur_tile_count(p, kMaskBlurZc)) + align_up(vol_t_tile_count(p));
            L.part_s = std::max(L.part_s, (size_t)ns);
            L.part_v = std::max(L.part_v, (size_t)nv);
        }
        if (b2d) {
            // room for the largest item lists of every 2D work shape the tuner may pick
            const Geo2D g = plan_geo2d(p, 0, 0);
            std::vector<int4> c;
            size_t na = 0, nb = 0;
            for (const Tiles2D &t : tiles2d_candidates()) {
                std::vector<int4> a, b;
                append_items_bp2d(g, 0, a, t);
                append_items_fp2d(g, 0, b, t);
                na = std::max(na, a.size());
                nb = std::max(nb, b.size());
            }
            append_items_tr2d(g, 0, c);
            L.max_items_bp += (int)na;
            L.max_items_fp += (int)nb;
            L.max_items_tr += (int)c.size();
        }
    }
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t r = off; off += align_up(bytes); return r; };
    const size_t sb = (size_t)L.NS * L.eb, vb = (size_t)L.NV * L.eb;
    L.y = take(sb); L.q = take(sb); L.Tj = take(sb); L.yt = take(sb); L.y0 = take(sb); L.ylast = take(sb);
    L.act = take((size_t)L.NS);
    L.lu = take(vb); L.ll = take(vb); L.D = take(vb); L.Dt = take(vb); L.D0 = take(vb); L.z = take(vb);
    L.tmp = take(vb); L.tmp2 = take(vb); L.s_up = take(vb); L.s_lo = take(vb); L.lut = take(vb); L.llt = take(vb);
    L.luo = take(vb); L.llo = take(vb); L.snap_u = take(vb); L.snap_l = take(vb); L.lu0 = take(vb); L.ll0 = take(vb);
    L.lul = take(vb); L.lll = take(vb);
    L.lab = take((size_t)L.NV);
    L.lo = L.lohi ? take(vb) : 0;
    L.hi = L.lohi ? take(vb) : 0;
    // the projector's z-contiguous input, one per instance: in masked solves the parts of it that
    // stay zero are written once (setup) and then skipped
    L.vol_t = take(vb);
    L.pflags = take(L.pf_bytes);
    L.bflags = take(L.bf_bytes);
    L.psteps = take(L.ps_bytes);
    L.pcount = take(L.pc_bytes);
    L.pitems = take(L.pc_bytes);
    L.pqueue = take((size_t)kQueueStride * B);
    L.preach = take(L.reach_bytes);
    L.bneed = take(L.bn_bytes);
    L.kflags = take(L.kf_bytes);
    L.ppart = take(L.part_s * L.eb * kMaxSplitP);
    L.bpart = take(L.part_v * L.eb * kMaxSplitB);
    const int max_seg = std::max(std::max(L.max_seg_s, L.max_seg_v), 1);
    L.partials = take(sizeof(double) * kNS * max_seg);
    L.insts = take(sizeof(InstC) * B);
    L.scal = take(sizeof(DevScal) * B);
    L.segS = take(sizeof(Seg) * std::max(L.max_seg_s, 1));
    L.segV = take(sizeof(Seg) * std::max(L.max_seg_v, 1));
    L.firstS = take(sizeof(int) * B); L.cntS = take(sizeof(int) * B);
    L.firstV = take(sizeof(int) * B); L.cntV = take(sizeof(int) * B);
    L.segSL = take(sizeof(Seg) * std::max(L.max_seg_s, 1));
    L.segVL = take(sizeof(Seg) * std::max(L.max_seg_v, 1));
    L.firstVL = take(sizeof(int) * B); L.cntVL = take(sizeof(int) * B);
    L.live = take((size_t)L.max_seg_s + L.max_seg_v + 2);
    L.list_act = take(sizeof(int) * B); L.list_tmp = take(sizeof(int) * B);
    L.sums = take(sizeof(double) * kNS * B);
    L.geo = take(sizeof(Geo2D) * B);
    L.items_bp = take(sizeof(int4) * std::max(L.max_items_bp, 1));
    L.items_fp = take(sizeof(int4) * std::max(L.max_items_fp, 1));
    L.items_tr = take(sizeof(int4) * std::max(L.max_items_tr, 1));
    L.total = off;
    return L;
}

struct Kkt {
    double eps_p = 0, eps_d = 0, eps_gap = 0, p = 0, d = 0, r_p = 0, r_d = 0;
    double rel() const { return std::max(eps_p, std::max(eps_d, eps_gap)); }
    double merit() const { return std::sqrt(eps_p * eps_p + eps_d * eps_d + eps_gap * eps_gap); }
};

template <typename T>
class Solver {
  public:
    Solver(const sipo_problem *probs, int B, const sipo_pdhg_options &o, char *ws, const Layout &L, hipStream_t s)
        : probs_(probs), B_(B), o_(o), ws_(ws), L_(L), s_(s) {
        b2d_ = use_batch2d(probs, B);
        in_.resize(B);
        hin_.resize(B);
        hsc_.resize(B);
        for (int i = 0; i < B; ++i) {
            const sipo_problem &pb = probs[i];
            Inst &I = in_[i];
            I.p = pb.plan;
            I.t3 = pb.plan->fast3d();
            I.ns = (long long)pb.plan->sino_elems();
            I.nv = (long long)pb.plan->vol_elems();
            I.soff = L.soff[i];
            I.voff = L.voff[i];
            InstC &c = hin_[i];
            std::memset(&c, 0, sizeof(c));
            c.c.u_free = pb.u_free;
            c.c.v_free = pb.v_free;
            c.c.w1 = pb.w1;
            c.c.w2 = pb.w2;
            c.c.h = pb.band_cap;
            c.c.lo_s = pb.lo_scalar;
            c.c.hi_s = pb.hi_scalar;
            c.c.wu = 1.0;
            c.c.wv = 1.0;
        }
    }
    ~Solver() {
        for (auto &e : zc_saved_) {
            e.p->p3d_zc = e.p3d;
            e.p->bp3d_zc = e.bp3d;
            e.p->blur_zc = e.blur;
            e.p->p3d_skip = e.skip;
        }
        if (graph_exec_) (void)hipGraphExecDestroy(graph_exec_);
        for (hipEvent_t e : ev_) (void)hipEventDestroy(e);
        for (hipEvent_t e : loop_ev_)
            if (e) (void)hipEventDestroy(e);
    }

    int run(sipo_pdhg_result *res);

  private:
    struct Inst {
        sipo_plan p;
        bool t3;
        long long ns, nv, soff, voff;
        double Tu = 0, Tv = 0, h_norm = 0, c_norm = 0;
        double omega = 1.0, m_anchor = 0, m_prev = 1e300, last_u = 0, last_v = 0, tau = 0, sigma = 0;
        int k_restart = 0, restarts = 0, iters = 0, status = SIPO_ITER_LIMIT;
        bool done = false;
        double fk = INFINITY;   // smallest Farkas violation of this check's candidates (progress lines)
        int cert = -1;      // certificate when infeasible: 0 / 1 iterate pairs, 2 the warm-start multipliers,
                            // 3 lambda(t), 4 lambda(t) - lambda at the last restart
        Kkt kc;
    };
    const sipo_problem *probs_;
    int B_;
    sipo_pdhg_options o_;
    char *ws_;
    const Layout &L_;
    hipStream_t s_;
    bool b2d_ = false;
    bool mask_ = false;                     // 3D operators skip workgroups the LP does not read
    bool masked_run_ = false;               // the iterations ran masked (mask_ ends before the last dose)
    std::vector<SplitSpec> psp_, bsp_;      // per instance: splits of the masked 3D operators
    std::vector<char> fused_;               // per instance: primal step fused into the masked projector
    std::vector<char> steps_;               // per instance: the masked projector walks its step lists
    // the plans' own slices per thread, which the masked operators change and the solver restores
    struct ZcSaved {
        sipo_plan p;
        int p3d, bp3d, blur;
        bool skip;
    };
    std::vector<ZcSaved> zc_saved_;
    int nc_max_ = 3;
    bool bp_staged_ = true;
    Tiles2D t2d_;                           // work shapes of the batched 2D pair
    int n_max_ = 1;
    std::vector<Inst> in_;
    std::vector<InstC> hin_;
    std::vector<DevScal> hsc_;
    std::vector<int> active_;               // instances the iteration kernels run on
    int n_seg_s_ = 0, n_seg_v_ = 0, n_items_bp_ = 0, n_items_fp_ = 0, n_items_tr_ = 0;
    // Segments where the primal step (some active ray) and the dual step (some labelled voxel, when
    // the dual step skips unlabelled ones) have work: per instance and segment, empty = all.  The
    // masks are fixed for the solve, so these are found once; the two steps launch over them only.
    std::vector<std::vector<uint8_t>> live_s_, live_v_;
    std::vector<int> fs_, cs_, fv_, cv_;   // ranges of each instance in the current full tables
    int n_seg_sl_ = 0, n_seg_vl_ = 0;
    std::vector<double> hsums_;             // [B][kNS]
    hipGraphExec_t graph_exec_ = nullptr;
    int graph_len_ = 0;
    // start and end of the iteration loop on the solve's stream: the start is recorded just before
    // the first iteration launch (after the first graph instantiation), the end after the last check
    hipEvent_t loop_ev_[2] = {nullptr, nullptr};
    bool loop_started_ = false;
    int mark_loop_start() {
        if (loop_started_) return SIPO_OK;
        SIPO_HIP(hipEventRecord(loop_ev_[0], s_));
        loop_started_ = true;
        return SIPO_OK;
    }

    // ---- typed views of the workspace
    T *F(size_t off) const { return (T *)(ws_ + off); }
    // a field or, for kNoField, NULL (the candidate and certificate kernels read it as zeros)
    const T *Fz(size_t off) const { return off == kNoField ? nullptr : (const T *)(ws_ + off); }
    uint8_t *U8(size_t off) const { return (uint8_t *)(ws_ + off); }
    template <typename X>
    X *P(size_t off) const { return (X *)(ws_ + off); }
    const T *lo_() const { return L_.lohi ? F(L_.lo) : nullptr; }
    const T *hi_() const { return L_.lohi ? F(L_.hi) : nullptr; }
    const Seg *segS() const { return P<Seg>(L_.segS); }
    const Seg *segV() const { return P<Seg>(L_.segV); }
    const Seg *segSL() const { return P<Seg>(L_.segSL); }
    // blur tile flags of a 3D instance (restarted solves): tiles holding a labelled voxel, and tiles
    // within the PSF radius of one
    uint8_t *blur_own(int i) const { return U8(L_.kflags) + L_.kfo[i]; }
    uint8_t *blur_reach(int i) const { return U8(L_.kflags) + L_.kfo[i] + align_up(blur_tile_count(in_[i].p, kMaskBlurZc)); }
    // transpose tiles of the projector's input that hold a voxel of a reach tile
    uint8_t *vol_t_on(int i) const { return blur_reach(i) + align_up(blur_tile_count(in_[i].p, kMaskBlurZc)); }
    const Seg *segVL() const { return P<Seg>(L_.segVL); }
    double *partials() const { return P<double>(L_.partials); }
    const InstC *insts() const { return P<InstC>(L_.insts); }
    DevScal *scal() const { return P<DevScal>(L_.scal); }

    int upload(size_t off, const void *src, size_t bytes) {
        if (!bytes) return SIPO_OK;
        SIPO_HIP(hipMemcpyAsync(ws_ + off, src, bytes, hipMemcpyHostToDevice, s_));
        SIPO_HIP(hipStreamSynchronize(s_));   // host staging may change right after
        return SIPO_OK;
    }
    int put_insts() { return upload(L_.insts, hin_.data(), sizeof(InstC) * B_); }
    int put_scal() { return upload(L_.scal, hsc_.data(), sizeof(DevScal) * B_); }
    int get_scal() {
        SIPO_HIP(hipMemcpyAsync(hsc_.data(), scal(), sizeof(DevScal) * B_, hipMemcpyDeviceToHost, s_));
        SIPO_HIP(hipStreamSynchronize(s_));
        return SIPO_OK;
    }
    void set_flags(const std::vector<int> &on) {
        for (int i = 0; i < B_; ++i) hin_[i].flag = 0;
        for (int i : on) hin_[i].flag = 1;
    }

    // Finds the segments with work for the primal and dual steps (see live_s_) and rebuilds the tables.
    int live_tables() {
        const size_t nv_off = (size_t)L_.max_seg_s;
        if (n_seg_s_)
            hipLaunchKernelGGL(k_seg_live, dim3(n_seg_s_), dim3(kThreads), 0, s_, (const uint8_t *)U8(L_.act), segS(),
                               U8(L_.live));
        if (mask_ && n_seg_v_)
            hipLaunchKernelGGL(k_seg_live, dim3(n_seg_v_), dim3(kThreads), 0, s_, (const uint8_t *)U8(L_.lab), segV(),
                               U8(L_.live) + nv_off);
        std::vector<uint8_t> h(nv_off + (size_t)L_.max_seg_v);
        SIPO_HIP(hipMemcpyAsync(h.data(), U8(L_.live), h.size(), hipMemcpyDeviceToHost, s_));
        SIPO_HIP(hipStreamSynchronize(s_));
        live_s_.assign(B_, {});
        live_v_.assign(B_, {});
        for (int i : active_) {
            live_s_[i].assign(h.begin() + fs_[i], h.begin() + fs_[i] + cs_[i]);
            if (mask_) live_v_[i].assign(h.begin() + nv_off + fv_[i], h.begin() + nv_off + fv_[i] + cv_[i]);
        }
        const std::vector<int> list = active_;
        return set_active(list);
    }

    // Segment tables, per-instance workgroup ranges and work items for the instances in `list`.
    int set_active(const std::vector<int> &list) {
        active_ = list;
        if (graph_exec_) {
            SIPO_HIP(hipGraphExecDestroy(graph_exec_));
            graph_exec_ = nullptr;
        }
        std::vector<Seg> ss, sv;
        std::vector<int> fs(B_, 0), cs(B_, 0), fv(B_, 0), cv(B_, 0);
        std::vector<int4> ib, ifp, itr;
        std::vector<Geo2D> geo(B_);
        nc_max_ = 3;
        n_max_ = 1;
        bp_staged_ = true;
        for (int i : list) {
            const Inst &I = in_[i];
            fs[i] = (int)ss.size();
            for (long long b = 0; b < I.ns; b += kChunk) ss.push_back({i, 0, I.soff + b, I.soff + std::min(I.ns, b + kChunk)});
            cs[i] = (int)ss.size() - fs[i];
            fv[i] = (int)sv.size();
            for (long long b = 0; b < I.nv; b += kChunk) sv.push_back({i, 0, I.voff + b, I.voff + std::min(I.nv, b + kChunk)});
            cv[i] = (int)sv.size() - fv[i];
            if (b2d_) {
                geo[i] = plan_geo2d(I.p, I.soff, I.voff);
                append_items_bp2d(geo[i], i, ib, t2d_);
                append_items_fp2d(geo[i], i, ifp, t2d_);
                append_items_tr2d(geo[i], i, itr);
                nc_max_ = std::max(nc_max_, I.p->p3d_nc);
                bp_staged_ = bp_staged_ && bp2d_stage_fits(I.p->n, I.p->n_bins, t2d_);
                n_max_ = std::max(n_max_, I.p->n);
            }
        }
        n_seg_s_ = (int)ss.size();
        n_seg_v_ = (int)sv.size();
        std::vector<Seg> ssl, svl;
        std::vector<int> fvl(B_, 0), cvl(B_, 0);
        for (int i : list) {
            const bool all_s = live_s_.empty() || live_s_[i].empty(), all_v = live_v_.empty() || live_v_[i].empty();
            const bool fused = !fused_.empty() && fused_[i];   // its primal step runs in the projector
            for (int k = 0; k < cs[i] && !fused; ++k)
                if (all_s || live_s_[i][k]) ssl.push_back(ss[fs[i] + k]);
            fvl[i] = (int)svl.size();
            for (int k = 0; k < cv[i]; ++k)
                if (all_v || live_v_[i][k]) svl.push_back(sv[fv[i] + k]);
            cvl[i] = (int)svl.size() - fvl[i];
        }
        n_seg_sl_ = (int)ssl.size();
        n_seg_vl_ = (int)svl.size();
        fs_ = fs; cs_ = cs; fv_ = fv; cv_ = cv;
        n_items_bp_ = (int)ib.size();
        n_items_fp_ = (int)ifp.size();
        n_items_tr_ = (int)itr.size();
        int rc = upload(L_.segS, ss.data(), sizeof(Seg) * ss.size());
        if (!rc) rc = upload(L_.segV, sv.data(), sizeof(Seg) * sv.size());
        if (!rc) rc = upload(L_.firstS, fs.data(), sizeof(int) * B_);
        if (!rc) rc = upload(L_.cntS, cs.data(), sizeof(int) * B_);
        if (!rc) rc = upload(L_.firstV, fv.data(), sizeof(int) * B_);
        if (!rc) rc = upload(L_.cntV, cv.data(), sizeof(int) * B_);
        if (!rc) rc = upload(L_.segSL, ssl.data(), sizeof(Seg) * ssl.size());
        if (!rc) rc = upload(L_.segVL, svl.data(), sizeof(Seg) * svl.size());
        if (!rc) rc = upload(L_.firstVL, fvl.data(), sizeof(int) * B_);
        if (!rc) rc = upload(L_.cntVL, cvl.data(), sizeof(int) * B_);
        if (!rc) rc = upload(L_.list_act, list.data(), sizeof(int) * list.size());
        if (!rc && b2d_) {
            rc = upload(L_.geo, geo.data(), sizeof(Geo2D) * B_);
            if (!rc) rc = upload(L_.items_bp, ib.data(), sizeof(int4) * ib.size());
            if (!rc) rc = upload(L_.items_fp, ifp.data(), sizeof(int4) * ifp.size());
            if (!rc) rc = upload(L_.items_tr, itr.data(), sizeof(int4) * itr.size());
        }
        return rc;
    }

    // Per-instance totals of the last reduction launched over the sinogram (S) or volume (V)
    // tables, for the instances in `list`; results in hsums_[i * kNS + k].
    int finish(bool vol, const std::vector<int> &list, int ns, bool max = false) {
        if (list.empty()) return SIPO_OK;
        int rc = upload(L_.list_tmp, list.data(), sizeof(int) * list.size());
        if (rc) return rc;
        const int *first = P<int>(vol ? L_.firstV : L_.firstS), *count = P<int>(vol ? L_.cntV : L_.cntS);
        if (max)
            hipLaunchKernelGGL(k_finish<true>, dim3(list.size()), dim3(kThreads), 0, s_, partials(), first, count,
                               P<int>(L_.list_tmp), ns, P<double>(L_.sums));
        else
            hipLaunchKernelGGL(k_finish<false>, dim3(list.size()), dim3(kThreads), 0, s_, partials(), first, count,
                               P<int>(L_.list_tmp), ns, P<double>(L_.sums));
        SIPO_HIP(hipMemcpyAsync(hsums_.data(), P<double>(L_.sums), sizeof(double) * kNS * B_, hipMemcpyDeviceToHost,
                                s_));
        SIPO_HIP(hipStreamSynchronize(s_));
        return SIPO_OK;
    }
    double sum(int i, int k) const { return hsums_[(size_t)i * kNS + k]; }

    // ---- streaming launches over the active tables
    dim3 gS() const { return dim3(std::max(n_seg_s_, 1)); }
    dim3 gV() const { return dim3(std::max(n_seg_v_, 1)); }
    void copyV(size_t dst, size_t src, bool flagged) {
        if (n_seg_v_) hipLaunchKernelGGL((k_copy<T>), gV(), dim3(kThreads), 0, s_, F(dst), (const T *)F(src), insts(),
                                         segV(), flagged ? 1 : 0);
    }
    void copyS(size_t dst, size_t src, bool flagged) {
        if (n_seg_s_) hipLaunchKernelGGL((k_copy<T>), gS(), dim3(kThreads), 0, s_, F(dst), (const T *)F(src), insts(),
                                         segS(), flagged ? 1 : 0);
    }
    int fill_vol(size_t dst) {   // zero a packed volume field over every instance
        const long long n = L_.NV;
        const int grid = (int)std::max<long long>(1, std::min<long long>((n + 255) / 256, 8192));
        hipLaunchKernelGGL((k_fill<T>), dim3(grid), dim3(256), 0, s_, F(dst), n, (T)0);
        return SIPO_OK;
    }
    int lambda_z(size_t lu, size_t ll, size_t z, bool flagged) {
        if (!n_seg_v_) return SIPO_OK;
        hipLaunchKernelGGL((k_lambda_z<T>), gV(), dim3(kThreads), 0, s_, F(lu), F(ll), F(z), U8(L_.lab), hi_(),
                           insts(), segV(), flagged ? 1 : 0, partials());
        return SIPO_OK;
    }

    // ---- operators on the solver's layouts (sinograms as held internally, volumes [z][y][x])
    int dose(size_t yf, size_t outf) {   // out = K P^T y on the active instances
        if (b2d_) {
            int rc = launch_bp2d(I_dtype(), bp_staged_, P<Geo2D>(L_.geo), P<int4>(L_.items_bp), n_items_bp_, F(yf),
                                 F(outf), 0, s_, t2d_);
            return rc ? rc : mark(SIPO_PHASE_BACKPROJECT);
        }
        for (int i : active_) {
            const Inst &I = in_[i];
            const T *y = F(yf) + I.soff;
            T *out = F(outf) + I.voff;
            const bool m = mask_ && I.t3;
            const uint8_t *on = m ? U8(L_.bflags) + L_.bfo[i] : nullptr;
            const SplitSpec sp = m ? bsp_[i] : SplitSpec();
            if (!I.p->has_psf) {
                int rc = launch_backproject_t(I.p, y, out, 0, s_, on, sp);
                if (!rc) rc = mark(SIPO_PHASE_BACKPROJECT);
                if (rc) return rc;
                continue;
            }
            T *tmp = F(L_.tmp) + I.voff;
            // masked: switched-off tiles of tmp keep older (finite) values; the blur reads them only
            // in halos of outputs the solve does not read (tmp is zeroed at setup)
            SplitSpec spk = sp;
            spk.keep_off = m;
            int rc = launch_backproject_t(I.p, y, tmp, 0, s_, on, spk);
            if (!rc) rc = mark(SIPO_PHASE_BACKPROJECT);
            // masked: the dose is read on labelled voxels only, so tiles without one are skipped
            if (!rc) rc = launch_blur(I.p, tmp, out, s_, m ? blur_own(i) : nullptr, 0);
            if (!rc) rc = mark(SIPO_PHASE_BLUR);
            if (rc) return rc;
        }
        return SIPO_OK;
    }
    // out = P K z on the active instances; with fuse_primal, instances whose primal step is fused
    // into the projector take that step instead (y, t.y updated; out not written for them)
    int adjoint(size_t zf, size_t outf, bool fuse_primal = false) {
        if (b2d_) {
            // rays marching along x read an [x][y] copy (tmp is free: no blur in this path)
            int rc = launch_tr2d(I_dtype(), P<Geo2D>(L_.geo), P<int4>(L_.items_tr), n_items_tr_, F(zf), F(L_.tmp), s_);
            if (!rc) rc = mark(SIPO_PHASE_TRANSPOSE);
            if (!rc) rc = launch_fp2d(I_dtype(), nc_max_, n_max_, P<Geo2D>(L_.geo), P<int4>(L_.items_fp), n_items_fp_, F(zf),
                                      F(L_.tmp), F(outf), 0, s_, t2d_);
            return rc ? rc : mark(SIPO_PHASE_PROJECT);
        }
        for (int i : active_) {
            const Inst &I = in_[i];
            const T *src = F(zf) + I.voff;
            T *out = F(outf) + I.soff;
            int rc = SIPO_OK;
            bool in_t = false;   // src is already in the projector's layout
            if (I.p->has_psf) {
                // masked: z vanishes off the labelled voxels, so K z is zero on tiles out of the PSF's
                // reach of them; those tiles are written as zeros without reading z, or (FP32) the
                // blur writes the projector's layout itself, where they stay zero from setup on
                const bool m = mask_ && I.t3;
                if (m && blur_to_t_ok(I.p)) {
                    T *vt = F(L_.vol_t) + I.voff;
                    rc = launch_blur_to_t(I.p, src, vt, s_, blur_reach(i));
                    src = vt;
                    in_t = true;
                } else {
                    T *tmp = F(L_.tmp) + I.voff;
                    rc = launch_blur(I.p, src, tmp, s_, m ? blur_reach(i) : nullptr, 1);
                    src = tmp;
                }
                if (!rc) rc = mark(SIPO_PHASE_BLUR);
            }
            if (!rc && I.t3 && !in_t) {
                // masked: only tiles that can hold a nonzero of K z (with a PSF; without one, z's own
                // support is not tracked per tile and the whole volume moves)
                const bool mt = mask_ && I.p->has_psf;
                T *vt = F(L_.vol_t) + I.voff;
                rc = launch_vol_to_t(I.p, src, vt, s_, mt ? vol_t_on(i) : nullptr);
                if (!rc) rc = mark(SIPO_PHASE_TRANSPOSE);
                src = vt;
            }
            if (!rc) {
                const bool m = mask_ && I.t3;
                PrimalFuse fz;
                const bool fuse = fuse_primal && m && !fused_.empty() && fused_[i];
                if constexpr (sizeof(T) == 4) {
                    if (fuse) {
                        fz.y = F(L_.y) + I.soff;
                        fz.yt = F(L_.yt) + I.soff;
                        fz.Tj = F(L_.Tj) + I.soff;
                        fz.y0 = F(L_.y0) + I.soff;
                        fz.act = U8(L_.act) + I.soff;
                        fz.tau_fac = &scal()[i].tau_fac;
                        fz.w_rho = &scal()[i].w;
                    }
                }
                const StepList sl = m ? step_list(i, false) : StepList();
                rc = launch_project_t(I.p, src, out, s_, m ? U8(L_.pflags) + L_.pfo[i] : nullptr,
                                      m ? psp_[i] : SplitSpec(), fuse ? &fz : nullptr, sl);
            }
            if (!rc) rc = mark(SIPO_PHASE_PROJECT);
            if (rc) return rc;
        }
        return SIPO_OK;
    }
    sipo_dtype I_dtype() const { return sizeof(T) == 8 ? SIPO_F64 : SIPO_F32; }

    // ---- masked 3D operators: per-instance skip flags, step lists and splits for the plan's
    // current slice counts.  bparts > 0 fixes the backprojector's view splits; 0 takes the rule:
    // enough parts that the switched-on tiles give about four workgroups per CU.  The projector's
    // march is split only when fewer of its workgroups stay on than there are CUs.
    int cus_ = 256;
    int mask_setup(int i, int bparts) {
        const Inst &I = in_[i];
        sipo_plan p = I.p;
        auto count_on = [&](size_t flags_off, size_t count) -> long long {
            std::vector<uint8_t> h(count);
            if (count && hipMemcpyAsync(h.data(), U8(flags_off), count, hipMemcpyDeviceToHost, s_) != hipSuccess)
                return -1;
            if (hipStreamSynchronize(s_) != hipSuccess) return -1;
            long long on = 0;
            for (uint8_t f : h) on += f ? 1 : 0;
            return on;
        };
        auto parts_for = [&](long long on, long long want, int max_parts) {
            if (on <= 0) return 1;
            return (int)std::min<long long>(max_parts, std::max<long long>(1, (want + on - 1) / on));
        };
        int rc = launch_p3d_flags(p, U8(L_.act) + I.soff, U8(L_.pflags) + L_.pfo[i], s_);
        if (!rc) rc = launch_bp3d_flags(p, U8(L_.lab) + I.voff, U8(L_.bflags) + L_.bfo[i], s_);
        if (!rc) rc = launch_bp3d_need(p, U8(L_.lab) + I.voff, U8(L_.preach), U8(L_.bneed) + L_.bno[i], s_);
        if (!rc) rc = launch_blur_flags(p, U8(L_.lab) + I.voff, blur_own(i), blur_reach(i), s_);
        if (!rc) rc = launch_vol_t_flags(p, blur_reach(i), vol_t_on(i), s_);
        if (rc) return rc;
        // the asynchronous projector walks only the march steps that can meet K z (FP32)
        steps_[i] = 0;
        if (sizeof(T) == 4 && p3d_steps_ok(p)) {
            rc = launch_p3d_steps(p, U8(L_.lab) + I.voff, U8(L_.pflags) + L_.pfo[i], U8(L_.preach),
                                  P<int>(L_.psteps + L_.pso[i]), P<int>(L_.pcount + L_.pco[i]), s_);
            if (rc) return rc;
            steps_[i] = 1;
        }
        const long long onp = count_on(L_.pflags + L_.pfo[i], p3d_flag_count(p));
        const long long onb = count_on(L_.bflags + L_.bfo[i], bp3d_flag_count(p));
        if (onp < 0 || onb < 0) return fail(SIPO_E_DEVICE, "pdhg setup: reading the skip flags failed");
        psp_[i] = SplitSpec{parts_for(onp, cus_, kMaxSplitP), F(L_.ppart)};
        pon_[i] = onp;
        bsp_[i] = SplitSpec{bparts > 0 ? std::min(bparts, kMaxSplitB) : parts_for(onb, 4LL * cus_, kMaxSplitB),
                            F(L_.bpart)};
        bsp_[i].need = U8(L_.bneed) + L_.bno[i];
        // the primal step rides in the projector's output when its march is not split (FP32), unless
        // it is set to run as its own kernel
        fused_[i] = sizeof(T) == 4 && p->p3d_dma && psp_[i].parts == 1 && pfuse_[i] >= 0;
        // the unsplit listed march takes its switched-on workgroups from a queue, longest list first
        n_pitems_[i] = 0;
        if (steps_[i] && psp_[i].parts == 1) {
            const size_t cnt = p3d_flag_count(p);
            std::vector<int> hc(cnt);
            std::vector<uint8_t> hf(cnt);
            if (cnt && (hipMemcpyAsync(hc.data(), P<int>(L_.pcount + L_.pco[i]), sizeof(int) * cnt,
                                       hipMemcpyDeviceToHost, s_) != hipSuccess ||
                        hipMemcpyAsync(hf.data(), U8(L_.pflags) + L_.pfo[i], cnt, hipMemcpyDeviceToHost, s_) !=
                            hipSuccess ||
                        hipStreamSynchronize(s_) != hipSuccess))
                return fail(SIPO_E_DEVICE, "pdhg setup: reading the projector's step counts failed");
            std::vector<int> items;
            for (size_t w = 0; w < cnt; ++w)
                if (hf[w]) items.push_back((int)w);
            std::stable_sort(items.begin(), items.end(), [&](int a, int b) { return hc[a] > hc[b]; });
            if (!items.empty()) {
                SIPO_HIP(hipMemcpyAsync(P<int>(L_.pitems + L_.pco[i]), items.data(), sizeof(int) * items.size(),
                                        hipMemcpyHostToDevice, s_));
                SIPO_HIP(hipMemsetAsync(U8(L_.pqueue) + kQueueStride * i, 0, 2 * sizeof(int), s_));
                SIPO_HIP(hipStreamSynchronize(s_));
            }
            n_pitems_[i] = (int)items.size();
        }
        return SIPO_OK;
    }
    std::vector<int> n_pitems_;   // per instance: tiles in the projector's work queue
    std::vector<long long> pon_;  // per instance: switched-on projector workgroups
    std::vector<int> pqueue_;     // per instance: queue workgroups per CU (-1 = one workgroup per tile)
    std::vector<int> pfuse_;      // per instance: -1 = the primal step runs as its own kernel
    StepList step_list(int i, bool off_unread) {
        StepList sl;
        if (steps_.empty() || !steps_[i]) return sl;
        sl.steps = P<int>(L_.psteps + L_.pso[i]);
        sl.count = P<int>(L_.pcount + L_.pco[i]);
        sl.n_on = pon_[i];
        sl.chunk = o_.op_config[7];
        if (n_pitems_[i] > 0 && pqueue_[i] > 0) {
            sl.items = P<int>(L_.pitems + L_.pco[i]);
            sl.n_items = n_pitems_[i];
            sl.queue = P<int>(L_.pqueue + kQueueStride * i);
            sl.queue_per_cu = pqueue_[i];
            sl.off_unread = off_unread;
        }
        return sl;
    }

    // Mean stream time (ms) of reps calls of fn after one untimed call.
    template <typename Fn>
    int time_launches(Fn fn, int reps, double &ms) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        SIPO_HIP(hipEventCreate(&e0));
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return fail(SIPO_E_DEVICE, "hipEventCreate failed");
        }
        int rc = fn();
        if (!rc) rc = hipEventRecord(e0, s_) == hipSuccess ? SIPO_OK : fail(SIPO_E_DEVICE, "hipEventRecord failed");
        for (int r = 0; r < reps && !rc; ++r) rc = fn();
        if (!rc) rc = hipEventRecord(e1, s_) == hipSuccess ? SIPO_OK : fail(SIPO_E_DEVICE, "hipEventRecord failed");
        float t = 0.f;
        if (!rc && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess))
            rc = fail(SIPO_E_DEVICE, "operator timing failed");
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        ms = t / reps;
        return rc;
    }

    // Work splits of the masked operators timed on this instance's own masks: the projector's slices
    // per thread, work queue and primal step, the backprojector's slices per thread and view splits,
    // and the blur's slices per chunk.  Candidates run in a fixed preference order and a later one
    // replaces the best only when it is more than 2 % faster, so near-ties resolve the same way from
    // run to run.  Inputs are the zeroed working fields: the operators' work does not depend on the
    // values.
    int tune_masked(int i, int &bparts) {
        const Inst &I = in_[i];
        sipo_plan p = I.p;
        constexpr int kReps = 3;
        double ms = 0;
        int rc = SIPO_OK;
        auto proj = [&]() {
            // as the iteration runs it: the primal step fused where it is fused there, else the primal
            // kernel after the projector, but writing fields that setup fills afterwards (q, T_j) instead
            // of y and t.y; timing only, so the queue's unwritten outputs of switched-off tiles are
            // never read
            PrimalFuse fz;
            const bool fuse = sizeof(T) == 4 && fused_[i];
            if constexpr (sizeof(T) == 4) {
                fz.y = F(L_.q) + I.soff;
                fz.yt = F(L_.Tj) + I.soff;
                fz.Tj = F(L_.Tj) + I.soff;
                fz.y0 = F(L_.y0) + I.soff;
                fz.act = U8(L_.act) + I.soff;
                fz.tau_fac = &scal()[i].tau_fac;
                fz.w_rho = &scal()[i].w;
            }
            int r = launch_project_t(p, F(L_.vol_t) + I.voff, F(L_.q) + I.soff, s_, U8(L_.pflags) + L_.pfo[i],
                                     psp_[i], fuse ? &fz : nullptr, step_list(i, true));
            if (!r && !fuse && n_seg_s_)
                hipLaunchKernelGGL((k_primal<T, true>), gS(), dim3(kThreads), 0, s_, F(L_.Tj), F(L_.Tj),
                                   (const T *)F(L_.q), (const T *)F(L_.Tj), (const uint8_t *)U8(L_.act),
                                   (const T *)F(L_.y0), (const DevScal *)scal(), segS());
            return r;
        };
        auto back = [&]() {
            SplitSpec sp = bsp_[i];
            sp.keep_off = p->has_psf;
            return launch_backproject_t(p, F(L_.yt) + I.soff, F(L_.tmp) + I.voff, 0, s_, U8(L_.bflags) + L_.bfo[i], sp);
        };
        auto blurs = [&]() {   // as the iteration runs them (the second into the projector's layout where it can)
            int r = launch_blur(p, F(L_.tmp) + I.voff, F(L_.Dt) + I.voff, s_, blur_own(i), 0);
            if (!r)
                r = blur_to_t_ok(p) ? launch_blur_to_t(p, F(L_.Dt) + I.voff, F(L_.vol_t) + I.voff, s_, blur_reach(i))
                                    : launch_blur(p, F(L_.Dt) + I.voff, F(L_.tmp2) + I.voff, s_, blur_reach(i), 1);
            return r;
        };
        // projector: 8, 16 or 32 slices per thread (the asynchronous variant only)
        const int *fx = o_.op_config;   // nonzero entries are fixed by the caller
        if (sizeof(T) == 4 && p->p3d_dma && p->nz % 4 == 0 && !fx[0]) {
            int best = p->p3d_zc, best_q = pqueue_[i], best_f = pfuse_[i];
            bool best_skip = p->p3d_skip;
            double best_ms = INFINITY;
            for (int zc : {16, 8, 32}) {
                if (zc > 8 && zc / 2 >= p->nz) continue;
                p->p3d_zc = zc;
                for (int pf : {1, -1}) {
                    if (fx[5] && pf != fx[5]) continue;
                    pfuse_[i] = pf;
                    rc = mask_setup(i, fx[2] ? fx[2] : bsp_[i].parts);
                    if (rc) return rc;
                    // skipping the LDS reads of out-of-reach candidates changes no result (their
                    // weights are zero), only the time
                    for (bool skip : {true, false}) {
                        if (fx[6] && skip != (fx[6] > 0)) continue;
                        p->p3d_skip = skip;
                        for (int qw : {-1, 3, 6, 16}) {   // 16: as many as fit
                            if (fx[4] && qw != fx[4]) continue;
                            pqueue_[i] = qw;
                            rc = time_launches(proj, kReps, ms);
                            if (rc) return rc;
                            if (ms < kTuneMargin * best_ms) {
                                best_ms = ms; best = zc; best_q = qw; best_f = pf; best_skip = skip;
                            }
                        }
                    }
                }
            }
            p->p3d_zc = best;
            p->p3d_skip = best_skip;
            pqueue_[i] = best_q;
            pfuse_[i] = best_f;
            tuned_.p_ms = best_ms;
        }
        // backprojector: 4, 8 or 16 slices per thread, each with 1, 2, 4 or 8 view splits
        {
            int best = p->bp3d_zc, best_parts = fx[2];
            double best_ms = INFINITY;
            for (int zc : {8, 4, 16}) {
                if (fx[1] ? zc != fx[1] : (zc > 4 && zc / 2 >= p->nz)) continue;
                p->bp3d_zc = zc;
                for (int parts : {8, 4, 2, 1}) {
                    if (fx[2] && parts != fx[2]) continue;
                    rc = mask_setup(i, parts);
                    if (!rc) rc = time_launches(back, kReps, ms);
                    if (rc) return rc;
                    if (ms < kTuneMargin * best_ms) { best_ms = ms; best = zc; best_parts = parts; }
                }
            }
            p->bp3d_zc = best;
            tuned_.bp_parts = best_parts;
            tuned_.bp_ms = best_ms;
        }
        // blur (both masked applications of an iteration): 4 or 8 slices per chunk
        if (p->has_psf && !fx[3]) {
            int best = p->blur_zc;
            double best_ms = INFINITY;
            for (int zc : {4, 8}) {
                if (zc > 4 && zc / 2 >= p->nz) break;
                p->blur_zc = zc;
                rc = mask_setup(i, tuned_.bp_parts);
                if (!rc) rc = time_launches(blurs, kReps, ms);
                if (rc) return rc;
                if (ms < kTuneMargin * best_ms) { best_ms = ms; best = zc; }
            }
            p->blur_zc = best;
            tuned_.k_ms = best_ms;
        }
        bparts = tuned_.bp_parts;
        if (o_.progress_every > 0)
            fprintf(stderr, "[sipo] instance %d: masked operators tuned: P %d slices/thread, %s, queue %d/CU, primal "
                    "step %s %.4f ms, P^T %d slices/thread x %d view splits %.4f ms, blur %d slices/chunk %.4f ms (both "
                    "applications)\n", i, p->p3d_zc, p->p3d_skip ? "skip" : "no skip", pqueue_[i],
                    pfuse_[i] > 0 ? "fused" : "separate", tuned_.p_ms, p->bp3d_zc, bparts, tuned_.bp_ms,
                    p->has_psf ? p->blur_zc : 0, tuned_.k_ms);
        return SIPO_OK;
    }
    // Work shapes of the batched 2D pair timed on this batch (FP32): the backprojector's tile (32 x 8,
    // 16 x 16, 64 x 4 voxels) and views per staged batch (16, 8, 32), then the projector's bundle (64,
    // 32, 128 bins); preference order and 2 % margin as for the 3D splits.  Caller-fixed shapes
    // (options tiles_2d) are kept.  Only shapes whose staged windows fit every instance are tried.
    int tune_2d() {
        constexpr int kReps = 3;
        const int *fx = o_.tiles_2d;
        std::vector<int> all(B_);
        for (int i = 0; i < B_; ++i) all[i] = i;
        auto fits = [&](const Tiles2D &t) {
            for (int i = 0; i < B_; ++i)
                if (!bp2d_stage_fits(in_[i].p->n, in_[i].p->n_bins, t)) return false;
            return true;
        };
        double ms = 0, best_ms = INFINITY;
        Tiles2D best = t2d_;
        int rc = SIPO_OK;
        if (!fx[0] && !fx[1]) {
            for (const Tiles2D &c : tiles2d_candidates()) {
                if (c.fb != t2d_.fb || !fits(c)) continue;
                Tiles2D t = t2d_;
                t.bx = c.bx; t.by = c.by; t.vb = c.vb;
                t2d_ = t;
                rc = set_active(all);
                if (!rc) rc = time_launches([&]() { return dose(L_.yt, L_.tmp2); }, kReps, ms);
                if (rc) return rc;
                if (ms < kTuneMargin * best_ms) { best_ms = ms; best = t; }
            }
            t2d_ = best;
            tuned_.bp_ms = best_ms;
        }
        if (!fx[2]) {
            best_ms = INFINITY;
            best = t2d_;
            for (int fb : {64, 32, 128}) {
                Tiles2D t = t2d_;
                t.fb = fb;
                t2d_ = t;
                rc = set_active(all);
                if (!rc) rc = time_launches([&]() { return adjoint(L_.lu, L_.q); }, kReps, ms);
                if (rc) return rc;
                if (ms < kTuneMargin * best_ms) { best_ms = ms; best = t; }
            }
            t2d_ = best;
            tuned_.p_ms = best_ms;
        }
        rc = set_active(all);
        if (!rc && o_.progress_every > 0)
            fprintf(stderr, "[sipo] 2D batch of %d: work shapes tuned: P^T %d x %d voxels, %d views per batch %.4f ms, "
                    "P %d bins x %d views %.4f ms\n", B_, t2d_.bx, t2d_.by, t2d_.vb, tuned_.bp_ms, t2d_.fb, t2d_.fv(),
                    tuned_.p_ms);
        return rc;
    }
    struct Tuned {
        int bp_parts = 0;
        double p_ms = 0, bp_ms = 0, k_ms = 0;
    } tuned_;

    // ---- profile mode: a timeline of events between consecutive iteration launches
    bool prof_on_ = false;
    std::vector<hipEvent_t> ev_;
    std::vector<int> ev_phase_;
    size_t ev_used_ = 0;
    double phase_ms_[SIPO_NUM_PHASES] = {};
    int phase_n_[SIPO_NUM_PHASES] = {};
    int mark(int phase) {
        if (!prof_on_) return SIPO_OK;
        if (ev_used_ == ev_.size()) {
            if (ev_.size() >= 4096) {
                int rc = flush_profile();
                if (rc) return rc;
            } else {
                hipEvent_t e;
                SIPO_HIP(hipEventCreate(&e));
                ev_.push_back(e);
                ev_phase_.push_back(-1);
            }
        }
        ev_phase_[ev_used_] = phase;
        SIPO_HIP(hipEventRecord(ev_[ev_used_], s_));
        ++ev_used_;
        return SIPO_OK;
    }
    int flush_profile() {
        if (ev_used_ == 0) return SIPO_OK;
        SIPO_HIP(hipEventSynchronize(ev_[ev_used_ - 1]));
        for (size_t i = 1; i < ev_used_; ++i) {
            const int ph = ev_phase_[i];
            if (ph < 0) continue;   // interval that starts a new timeline segment
            float ms = 0.f;
            SIPO_HIP(hipEventElapsedTime(&ms, ev_[i - 1], ev_[i]));
            phase_ms_[ph] += ms;
            phase_n_[ph] += 1;
        }
        ev_used_ = 0;
        return SIPO_OK;
    }

    int pack();
    int unpack();
    int setup_common();
    int power_norm(int iters, std::vector<double> &nrm);
    int kkt(size_t y, size_t D, bool at_t, size_t lu, size_t ll, size_t z, const std::vector<int> &list);
    int farkas(size_t alu, size_t all, size_t blu, size_t bll, double tol, const std::vector<int> &list,
               std::vector<char> &ok);
    int iteration(bool check);
    int run_block(int nblk);
};

// Copy the callers' arrays into the packed workspace (internal layout for 3D instances).
template <typename T>
int Solver<T>::pack() {
    for (int i = 0; i < B_; ++i) {
        const sipo_problem &pb = probs_[i];
        const Inst &I = in_[i];
        const size_t vb = (size_t)I.nv * sizeof(T), sb = (size_t)I.ns * sizeof(T);
        if (I.t3) {
            int rc = launch_sino_to_t(I.p, pb.y, F(L_.y) + I.soff, s_);
            if (!rc) rc = launch_mask_to_t(I.p, pb.act, U8(L_.act) + I.soff, s_);
            if (rc) return rc;
        } else {
            SIPO_HIP(hipMemcpyAsync(F(L_.y) + I.soff, pb.y, sb, hipMemcpyDeviceToDevice, s_));
            SIPO_HIP(hipMemcpyAsync(U8(L_.act) + I.soff, pb.act, (size_t)I.ns, hipMemcpyDeviceToDevice, s_));
        }
        SIPO_HIP(hipMemcpyAsync(F(L_.lu) + I.voff, pb.lam_up, vb, hipMemcpyDeviceToDevice, s_));
        SIPO_HIP(hipMemcpyAsync(F(L_.ll) + I.voff, pb.lam_lo, vb, hipMemcpyDeviceToDevice, s_));
        SIPO_HIP(hipMemcpyAsync(U8(L_.lab) + I.voff, pb.labels, (size_t)I.nv, hipMemcpyDeviceToDevice, s_));
        if (L_.lohi) {
            const int grid = (int)std::min<long long>((I.nv + 255) / 256, 4096);
            if (pb.lo) SIPO_HIP(hipMemcpyAsync(F(L_.lo) + I.voff, pb.lo, vb, hipMemcpyDeviceToDevice, s_));
            else hipLaunchKernelGGL((k_fill<T>), dim3(grid), dim3(256), 0, s_, F(L_.lo) + I.voff, I.nv, (T)pb.lo_scalar);
            if (pb.hi) SIPO_HIP(hipMemcpyAsync(F(L_.hi) + I.voff, pb.hi, vb, hipMemcpyDeviceToDevice, s_));
            else hipLaunchKernelGGL((k_fill<T>), dim3(grid), dim3(256), 0, s_, F(L_.hi) + I.voff, I.nv, (T)pb.hi_scalar);
        }
    }
    SIPO_LAUNCHED("pdhg pack");
    return SIPO_OK;
}

// Returned point and dose back to the callers' arrays.
template <typename T>
int Solver<T>::unpack() {
    for (int i = 0; i < B_; ++i) {
        const sipo_problem &pb = probs_[i];
        const Inst &I = in_[i];
        const size_t vb = (size_t)I.nv * sizeof(T), sb = (size_t)I.ns * sizeof(T);
        if (I.t3) {
            int rc = launch_sino_from_t(I.p, F(L_.y) + I.soff, pb.y, 0, s_);
            if (rc) return rc;
        } else {
            SIPO_HIP(hipMemcpyAsync(pb.y, F(L_.y) + I.soff, sb, hipMemcpyDeviceToDevice, s_));
        }
        SIPO_HIP(hipMemcpyAsync(pb.lam_up, F(L_.lu) + I.voff, vb, hipMemcpyDeviceToDevice, s_));
        SIPO_HIP(hipMemcpyAsync(pb.lam_lo, F(L_.ll) + I.voff, vb, hipMemcpyDeviceToDevice, s_));
        if (pb.dose_out) SIPO_HIP(hipMemcpyAsync(pb.dose_out, F(L_.D) + I.voff, vb, hipMemcpyDeviceToDevice, s_));
    }
    SIPO_LAUNCHED("pdhg unpack");
    return SIPO_OK;
}

// KKT of every instance in `list` at (y, D, lambda) with z = lambda_up - lambda_lo in field z;
// the scalars are t's (at_t) or z's.  Uses q as scratch; fills in_[i].kc.
template <typename T>
int Solver<T>::kkt(size_t yf, size_t Df, bool at_t, size_t luf, size_t llf, size_t zf, const std::vector<int> &list) {
    for (int i : list) {
        hin_[i].eu = at_t ? hsc_[i].ut_done : hsc_[i].u;
        hin_[i].ev = at_t ? hsc_[i].vt_done : hsc_[i].v;
    }
    int rc = put_insts();
    if (rc) return rc;
    hipLaunchKernelGGL((k_kkt_vox<T>), gV(), dim3(kThreads), 0, s_, (const T *)F(Df), (const T *)F(luf),
                       (const T *)F(llf), (const uint8_t *)U8(L_.lab), lo_(), hi_(), insts(), segV(), partials());
    rc = finish(true, list, 4);
    if (rc) return rc;
    std::vector<double> hv((size_t)B_ * 4);
    for (int i : list)
        for (int k = 0; k < 4; ++k) hv[(size_t)i * 4 + k] = sum(i, k);
    rc = adjoint(zf, L_.q);
    if (rc) return rc;
    hipLaunchKernelGGL((k_kkt_ray<T>), gS(), dim3(kThreads), 0, s_, (const T *)F(L_.q), (const T *)F(yf),
                       (const uint8_t *)U8(L_.act), segS(), partials());
    rc = finish(false, list, 2);
    if (rc) return rc;
    for (int i : list) {
        Inst &I = in_[i];
        const LPConst &c = hin_[i].c;
        const double u = hin_[i].eu, v = hin_[i].ev;
        const double *h4 = &hv[(size_t)i * 4];
        double rp2 = h4[0] + sum(i, 1);
        if (c.u_free && u < 0) rp2 += u * u;
        if (c.v_free && v < 0) rp2 += v * v;
        double rd2 = sum(i, 0);
        if (c.u_free) { const double r = c.w1 - h4[2]; if (r < 0) rd2 += r * r; }
        if (c.v_free) { const double r = c.w2 - h4[3]; if (r < 0) rd2 += r * r; }
        const double pobj = (c.u_free ? c.w1 * u : 0.0) + (c.v_free ? c.w2 * v : 0.0);
        double dobj = h4[1];
        if (!c.u_free) dobj -= c.h * h4[2];
        if (!c.v_free) dobj -= h4[3];
        Kkt &k = I.kc;
        k.r_p = std::sqrt(rp2);
        k.r_d = std::sqrt(rd2);
        k.eps_p = k.r_p / (1.0 + I.h_norm);
        k.eps_d = k.r_d / (1.0 + I.c_norm);
        k.eps_gap = std::fabs(pobj - dobj) / (1.0 + std::fabs(pobj) + std::fabs(dobj));
        k.p = pobj;
        k.d = dobj;
    }
    return SIPO_OK;
}

template <typename T>
int Solver<T>::setup_common() {
    int rc = pack();
    if (rc) return rc;
    std::vector<int> all(B_);
    for (int i = 0; i < B_; ++i) all[i] = i;
    rc = set_active(all);
    if (!rc) rc = put_insts();
    if (rc) return rc;
    hipLaunchKernelGGL((k_project_y<T>), gS(), dim3(kThreads), 0, s_, F(L_.y), (const uint8_t *)U8(L_.act), segS());
    copyS(L_.yt, L_.y, false);   // t.y starts as y: zero on masked rays, which the primal step never touches
    if (b2d_) {
        // the batched 2D pair's work shapes: fixed by the caller, tuned, or the defaults
        const int *fx = o_.tiles_2d;
        if (fx[0] || fx[1] || fx[2]) {
            if (fx[0]) { t2d_.bx = fx[0]; t2d_.by = 256 / fx[0]; }
            if (fx[1]) t2d_.vb = fx[1];
            if (fx[2]) t2d_.fb = fx[2];
            rc = set_active(all);
            if (rc) return rc;
        }
        if (o_.tune_operators && sizeof(T) == 4 && bp_staged_) {
            rc = tune_2d();
            if (rc) return rc;
        }
    }
    if (o_.mode == SIPO_PDHG_RESTARTED) {
        // From here on the 3D operators skip what the restarted scheme never reads: q = P K z off the
        // active rays, and P^T y away from the labelled voxels and their PSF neighbourhood (every row
        // scaling, residual and certificate test reads D on labelled voxels and q on active rays).
        // Few workgroups stay on, each with a long serial walk.  The masked projector runs with at most 16
        // slices per thread and the masked backprojector with at most 8 (finer chunks give more
        // workgroups; at 256^3 x 360 these are the fastest of the 4 / 8 / 16 / 32 choices), the
        // backprojector's view walk is split so that the switched-on tiles give about four workgroups
        // per CU, and the projector's march is split only when very few of its workgroups stay on.  The
        // plans' own settings are restored when the solver ends.
        cus_ = 256;
        (void)hipDeviceGetAttribute(&cus_, hipDeviceAttributeMultiprocessorCount, probs_[0].plan->device);
        psp_.assign(B_, SplitSpec());
        bsp_.assign(B_, SplitSpec());
        fused_.assign(B_, 0);
        steps_.assign(B_, 0);
        n_pitems_.assign(B_, 0);
        pon_.assign(B_, 0);
        pqueue_.assign(B_, o_.op_config[4] ? o_.op_config[4] : -1);
        pfuse_.assign(B_, o_.op_config[5] ? o_.op_config[5] : 1);
        for (int i = 0; i < B_; ++i) {
            const Inst &I = in_[i];
            if (!I.t3) continue;
            sipo_plan p = I.p;
            bool seen = false;
            for (auto &e : zc_saved_) seen = seen || e.p == p;
            if (!seen) {
                zc_saved_.push_back({p, p->p3d_zc, p->bp3d_zc, p->blur_zc, p->p3d_skip});
                p->blur_zc = o_.op_config[3] ? o_.op_config[3] : std::min(kMaskBlurZc, p->nz);
                p->p3d_zc = o_.op_config[0] ? o_.op_config[0] : std::min(p->p3d_zc, 16);
                p->bp3d_zc = o_.op_config[1] ? o_.op_config[1] : std::min(p->bp3d_zc, 8);
                if (o_.op_config[6]) p->p3d_skip = o_.op_config[6] > 0;
            }
            rc = mask_setup(i, o_.op_config[2]);
            if (rc) return rc;
        }
        mask_ = masked_run_ = true;
        fill_vol(L_.vol_t);   // zero where the masked transposes never write
        fill_vol(L_.tmp);     // finite where the masked backprojector leaves tiles as they are
        if (o_.tune_operators) {
            // tune on the first instance of each plan, then rebuild every instance's flags for the
            // plan's chosen slice counts (instances of one plan share them)
            struct Chosen { sipo_plan p; int parts, tuned_on; };   // plan, view splits, instance tuned on
            std::vector<Chosen> chosen;
            for (int i = 0; i < B_; ++i) {
                if (!in_[i].t3) continue;
                bool seen = false;
                for (auto &c : chosen) seen = seen || c.p == in_[i].p;
                if (seen) continue;
                int parts = 0;
                rc = tune_masked(i, parts);
                if (rc) return rc;
                chosen.push_back({in_[i].p, parts, i});
            }
            for (int i = 0; i < B_; ++i) {
                if (!in_[i].t3) continue;
                int parts = 0;
                for (auto &c : chosen)
                    if (c.p == in_[i].p) {
                        // the queue width and the primal step's form are per instance: take the tuned ones
                        parts = c.parts;
                        pqueue_[i] = pqueue_[c.tuned_on];
                        pfuse_[i] = pfuse_[c.tuned_on];
                    }
                rc = mask_setup(i, parts);
                if (rc) return rc;
            }
            fill_vol(L_.vol_t);
            fill_vol(L_.tmp);
        }
    }
    rc = live_tables();
    if (rc) return rc;
    rc = lambda_z(L_.lu, L_.ll, L_.z, false);
    if (!rc) rc = finish(true, all, 2);
    if (rc) return rc;
    std::vector<double> l1(B_), ul2(B_);
    for (int i = 0; i < B_; ++i) { l1[i] = sum(i, 0); ul2[i] = sum(i, 1); }
    // R = K P^T 1_act -> dual scalings; region sizes, ||h||
    hipLaunchKernelGGL((k_colweight<T>), gV(), dim3(kThreads), 0, s_, F(L_.tmp2), (const uint8_t *)U8(L_.lab), segV());
    hipLaunchKernelGGL((k_act_to_float<T>), gS(), dim3(kThreads), 0, s_, F(L_.q), (const uint8_t *)U8(L_.act), segS());
    rc = dose(L_.q, L_.Dt);
    if (rc) return rc;
    hipLaunchKernelGGL((k_row_scaling<T>), gV(), dim3(kThreads), 0, s_, (const T *)F(L_.Dt), F(L_.s_up), F(L_.s_lo),
                       (const uint8_t *)U8(L_.lab), lo_(), hi_(), insts(), segV(), partials());
    rc = finish(true, all, 6);
    if (rc) return rc;
    if (o_.mode == SIPO_PDHG_RESTARTED && o_.scalar_weight > 0) {
        // column weights of the free scalars: c times the mean row sum of their rows; redo the rows
        for (int i = 0; i < B_; ++i) {
            LPConst &c = hin_[i].c;
            if (sum(i, 0) > 0 && sum(i, 4) > 0) c.wu = o_.scalar_weight * sum(i, 4) / sum(i, 0);
            if (sum(i, 1) > 0 && sum(i, 5) > 0) c.wv = o_.scalar_weight * sum(i, 5) / sum(i, 1);
        }
        rc = put_insts();
        if (rc) return rc;
        hipLaunchKernelGGL((k_row_scaling<T>), gV(), dim3(kThreads), 0, s_, (const T *)F(L_.Dt), F(L_.s_up),
                           F(L_.s_lo), (const uint8_t *)U8(L_.lab), lo_(), hi_(), insts(), segV(), partials());
        rc = finish(true, all, 6);
        if (rc) return rc;
    }
    for (int i = 0; i < B_; ++i) {
        Inst &I = in_[i];
        const LPConst &c = hin_[i].c;
        I.Tu = (c.u_free && sum(i, 0) > 0) ? c.wu / sum(i, 0) : 0.0;
        I.Tv = (c.v_free && sum(i, 1) > 0) ? c.wv / sum(i, 1) : 0.0;
        I.h_norm = std::sqrt(sum(i, 2));
        I.c_norm = std::hypot(c.u_free ? c.w1 : 0.0, c.v_free ? c.w2 : 0.0);
    }
    // primal scaling T_j = 1 / (P K w)_j
    rc = adjoint(L_.tmp2, L_.Tj);
    if (rc) return rc;
    hipLaunchKernelGGL((k_inv_colsum<T>), gS(), dim3(kThreads), 0, s_, F(L_.Tj), (const uint8_t *)U8(L_.act), segS());
    rc = dose(L_.y, L_.D);
    if (rc) return rc;
    for (int i = 0; i < B_; ++i) {
        DevScal &h = hsc_[i];
        std::memset(&h, 0, sizeof(h));
        const LPConst &c = hin_[i].c;
        h.u = c.u_free ? std::max(0.0, probs_[i].u0) : c.h;
        h.v = c.v_free ? std::max(0.0, probs_[i].v0) : 1.0;
        h.init_l1 = l1[i];
        h.init_Ul2 = ul2[i];
    }
    return SIPO_OK;
}

// FP64 power iteration for ||G|| of every instance at once (plain mode).  Uses y0 as scratch.
template <typename T>
int Solver<T>::power_norm(int iters, std::vector<double> &nrm) {
    std::vector<int> all(B_);
    for (int i = 0; i < B_; ++i) all[i] = i;
    nrm.assign(B_, 0.0);
    const size_t y = L_.y0;
    hipLaunchKernelGGL((k_act_to_float<T>), gS(), dim3(kThreads), 0, s_, F(y), (const uint8_t *)U8(L_.act), segS());
    hipLaunchKernelGGL((k_pi_mask<T>), gS(), dim3(kThreads), 0, s_, F(y), (const T *)F(y), (const uint8_t *)U8(L_.act),
                       segS(), partials());
    int rc = finish(false, all, 1);
    if (rc) return rc;
    std::vector<double> u(B_), v(B_), lam(B_, 0.0);
    for (int i = 0; i < B_; ++i) {
        const LPConst &c = hin_[i].c;
        u[i] = c.u_free ? 1.0 : 0.0;
        v[i] = c.v_free ? 1.0 : 0.0;
        const double nr = std::sqrt(sum(i, 0) + u[i] * u[i] + v[i] * v[i]);
        if (!(nr > 0)) return fail(SIPO_E_INVALID, "instance %d: operator norm is zero (no active rays or regions)", i);
        hin_[i].fac = 1.0 / nr;
        u[i] /= nr;
        v[i] /= nr;
    }
    rc = put_insts();
    if (rc) return rc;
    hipLaunchKernelGGL((k_scale<T>), gS(), dim3(kThreads), 0, s_, F(y), insts(), segS());
    for (int it = 0; it < iters; ++it) {
        rc = dose(y, L_.Dt);
        if (rc) return rc;
        for (int i = 0; i < B_; ++i) { hin_[i].eu = u[i]; hin_[i].ev = v[i]; }
        rc = put_insts();
        if (rc) return rc;
        hipLaunchKernelGGL((k_pi_rows<T>), gV(), dim3(kThreads), 0, s_, (const T *)F(L_.Dt), F(L_.tmp2),
                           (const uint8_t *)U8(L_.lab), hi_(), insts(), segV(), partials());
        rc = finish(true, all, 2);
        if (rc) return rc;
        std::vector<double> rs0(B_), rs1(B_);
        for (int i = 0; i < B_; ++i) { rs0[i] = sum(i, 0); rs1[i] = sum(i, 1); }
        rc = adjoint(L_.tmp2, L_.q);
        if (rc) return rc;
        hipLaunchKernelGGL((k_pi_mask<T>), gS(), dim3(kThreads), 0, s_, F(y), (const T *)F(L_.q),
                           (const uint8_t *)U8(L_.act), segS(), partials());
        rc = finish(false, all, 1);
        if (rc) return rc;
        for (int i = 0; i < B_; ++i) {
            const LPConst &c = hin_[i].c;
            const double gu = c.u_free ? -rs0[i] : 0.0, gv = c.v_free ? -rs1[i] : 0.0;
            const double l = std::sqrt(sum(i, 0) + gu * gu + gv * gv);
            lam[i] = l;
            hin_[i].fac = l > 0 ? 1.0 / l : 1.0;
            u[i] = l > 0 ? gu / l : u[i];
            v[i] = l > 0 ? gv / l : v[i];
        }
        rc = put_insts();
        if (rc) return rc;
        hipLaunchKernelGGL((k_scale<T>), gS(), dim3(kThreads), 0, s_, F(y), insts(), segS());
    }
    for (int i = 0; i < B_; ++i) nrm[i] = std::sqrt(lam[i]);
    return SIPO_OK;
}

// Farkas test of d = max(a - b, 0) for the instances in `list`: scaled to dual objective 1,
// every reduced-cost violation must be <= tol.  Uses tmp2 (z_d) and q.
template <typename T>
int Solver<T>::farkas(size_t alu, size_t all, size_t blu, size_t bll, double tol, const std::vector<int> &list,
                      std::vector<char> &ok) {
    ok.assign(B_, 0);
    if (list.empty()) return SIPO_OK;
    set_flags(list);
    int rc = put_insts();
    if (rc) return rc;
    hipLaunchKernelGGL((k_ray_candidate<T>), gV(), dim3(kThreads), 0, s_, (const T *)F(alu), (const T *)F(all),
                       Fz(blu), Fz(bll), F(L_.tmp2), (const uint8_t *)U8(L_.lab), lo_(), hi_(), insts(), segV(),
                       partials());
    rc = finish(true, list, 4);
    if (rc) return rc;
    std::vector<int> need;
    std::vector<double> obj(B_, 0.0), sw(B_, 0.0);
    for (int i : list) {
        const LPConst &c = hin_[i].c;
        double ray_obj = sum(i, 0);
        if (!c.u_free) ray_obj -= c.h * sum(i, 1);
        if (!c.v_free) ray_obj -= sum(i, 2);
        if (!(ray_obj > 0) || !(sum(i, 3) > 0)) continue;
        const double worst_u = c.u_free ? sum(i, 1) / ray_obj : 0.0;
        const double worst_v = c.v_free ? sum(i, 2) / ray_obj : 0.0;
        const double ws = std::max(worst_u, worst_v);
        if (ws > tol) {
            in_[i].fk = std::min(in_[i].fk, ws);
            continue;
        }
        obj[i] = ray_obj;
        sw[i] = ws;
        need.push_back(i);
    }
    if (need.empty()) return SIPO_OK;
    rc = adjoint(L_.tmp2, L_.q);
    if (rc) return rc;
    hipLaunchKernelGGL((k_ray_check<T>), gS(), dim3(kThreads), 0, s_, (const T *)F(L_.q), (const uint8_t *)U8(L_.act),
                       segS(), partials());
    rc = finish(false, need, 2, true);
    if (rc) return rc;
    for (int i : need) {
        ok[i] = sum(i, 0) / obj[i] <= tol;
        in_[i].fk = std::min(in_[i].fk, std::max(sw[i], sum(i, 0) / obj[i]));
    }
    return SIPO_OK;
}

// One iteration of every active instance: t = T(z), z <- Halpern update.  On check
// iterations t.lambda and the pre-step lambda are written out.
template <typename T>
int Solver<T>::iteration(bool check) {
    const bool hal = o_.mode == SIPO_PDHG_RESTARTED;
    prof_on_ = o_.profile != 0;
    int rc = mark(-1);   // start of this iteration's timeline segment
    if (!rc) rc = adjoint(L_.z, L_.q, hal);
    if (rc) return rc;
    if (n_seg_sl_)
        hipLaunchKernelGGL((hal ? &k_primal<T, true> : &k_primal<T, false>), dim3(n_seg_sl_), dim3(kThreads), 0, s_,
                           F(L_.y), F(L_.yt), (const T *)F(L_.q), hal ? (const T *)F(L_.Tj) : (const T *)nullptr,
                           (const uint8_t *)U8(L_.act), hal ? (const T *)F(L_.y0) : (const T *)nullptr,
                           (const DevScal *)scal(), segSL());
    rc = mark(SIPO_PHASE_PRIMAL);
    if (!rc) rc = dose(L_.yt, L_.Dt);
    if (rc) return rc;
    if (n_seg_vl_)
        hipLaunchKernelGGL(dual_kernel<T>(hal, L_.lohi, mask_), dim3(n_seg_vl_), dim3(kThreads), 0, s_,
                           (const T *)F(L_.Dt), F(L_.D), hal ? (const T *)F(L_.D0) : (const T *)nullptr, F(L_.lu),
                           F(L_.ll), hal ? (const T *)F(L_.lu0) : (const T *)nullptr,
                           hal ? (const T *)F(L_.ll0) : (const T *)nullptr, F(L_.z), (const uint8_t *)U8(L_.lab), lo_(),
                           hi_(), hal ? (const T *)F(L_.s_up) : (const T *)nullptr,
                           hal ? (const T *)F(L_.s_lo) : (const T *)nullptr, check ? F(L_.lut) : (T *)nullptr,
                           check ? F(L_.llt) : (T *)nullptr, check ? F(L_.luo) : (T *)nullptr,
                           check ? F(L_.llo) : (T *)nullptr, (const DevScal *)scal(), insts(), segVL(), partials());
    rc = mark(SIPO_PHASE_DUAL);
    if (rc) return rc;
    hipLaunchKernelGGL(k_scalars, dim3(active_.size()), dim3(kThreads), 0, s_, (const double *)partials(),
                       (const int *)P<int>(L_.firstVL), (const int *)P<int>(L_.cntVL), (const int *)P<int>(L_.list_act),
                       scal(), insts());
    rc = mark(SIPO_PHASE_SCALARS);
    prof_on_ = false;
    return rc;
}

// nblk iterations, the last one a check iteration; captured once into a graph when requested
// (the graph stays valid while the active set does not change).
template <typename T>
int Solver<T>::run_block(int nblk) {
    if (!o_.use_graph) {
        int rc = mark_loop_start();
        if (rc) return rc;
        for (int j = 0; j < nblk; ++j) {
            rc = iteration(j == nblk - 1);
            if (rc) return rc;
        }
        SIPO_LAUNCHED("pdhg iteration");
        return SIPO_OK;
    }
    if (!graph_exec_ || graph_len_ != nblk) {
        if (graph_exec_) {
            SIPO_HIP(hipGraphExecDestroy(graph_exec_));
            graph_exec_ = nullptr;
        }
        hipGraph_t g = nullptr;
        SIPO_HIP(hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal));
        int rc = SIPO_OK;
        for (int j = 0; j < nblk && rc == SIPO_OK; ++j) rc = iteration(j == nblk - 1);
        hipError_t e = hipStreamEndCapture(s_, &g);
        if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
        if (e != hipSuccess) return fail(SIPO_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&graph_exec_, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return fail(SIPO_E_DEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
        graph_len_ = nblk;
    }
    int rc = mark_loop_start();
    if (rc) return rc;
    SIPO_HIP(hipGraphLaunch(graph_exec_, s_));
    return SIPO_OK;
}

template <typename T>
int Solver<T>::run(sipo_pdhg_result *res) {
    auto t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < B_; ++i) std::memset(&res[i], 0, sizeof(res[i]));
    hsums_.assign((size_t)B_ * kNS, 0.0);
    int rc = setup_common();
    if (rc) return rc;
    std::vector<int> all(B_);
    for (int i = 0; i < B_; ++i) all[i] = i;
    const bool hal = o_.mode == SIPO_PDHG_RESTARTED;
    const double eta = o_.eta > 0 ? o_.eta : 0.95;
    if (!hal) {
        std::vector<double> nrm;
        if (!(o_.tau > 0 && o_.sigma > 0)) {
            rc = power_norm(o_.power_iters > 0 ? o_.power_iters : 100, nrm);
            if (rc) return rc;
        }
        for (int i = 0; i < B_; ++i) {
            Inst &I = in_[i];
            if (o_.tau > 0 && o_.sigma > 0) { I.tau = o_.tau; I.sigma = o_.sigma; }
            else {
                if (!(nrm[i] > 0)) return fail(SIPO_E_INVALID, "instance %d: operator norm is zero", i);
                I.tau = I.sigma = 0.9 / nrm[i];
            }
            DevScal &h = hsc_[i];
            h.tau_fac = I.tau;
            h.sig_fac = I.sigma;
            h.tau_u = I.tau;
            h.tau_v = I.tau;
            h.halpern = 0.0;
            h.rho = 0.0;
        }
    } else {
        for (int i = 0; i < B_; ++i) {
            const Inst &I = in_[i];
            DevScal &h = hsc_[i];
            h.tau_fac = eta / I.omega;
            h.sig_fac = eta * I.omega;
            h.tau_u = eta * I.Tu / I.omega;
            h.tau_v = eta * I.Tv / I.omega;
            h.halpern = 1.0;
            h.rho = 1.0;
        }
    }
    for (int i = 0; i < B_; ++i) {
        hsc_[i].u0 = hsc_[i].u;
        hsc_[i].v0 = hsc_[i].v;
        in_[i].last_u = hsc_[i].u;
        in_[i].last_v = hsc_[i].v;
    }
    set_flags(all);
    rc = put_insts();
    if (!rc) rc = put_scal();
    if (rc) return rc;
    hipLaunchKernelGGL(k_scalars_init, dim3(1), dim3(kThreads), 0, s_, scal(), insts(), B_);
    if (hal) {
        // anchor, restart point and snapshot start at the initial point
        copyS(L_.y0, L_.y, false);
        copyS(L_.ylast, L_.y, false);
        copyV(L_.D0, L_.D, false);
        for (size_t dst : {L_.lu0, L_.lul, L_.snap_u}) copyV(dst, L_.lu, false);
        for (size_t dst : {L_.ll0, L_.lll, L_.snap_l}) copyV(dst, L_.ll, false);
        rc = get_scal();
        if (!rc) rc = kkt(L_.y, L_.D, false, L_.lu, L_.ll, L_.z, all);
        if (rc) return rc;
        for (int i = 0; i < B_; ++i) in_[i].m_anchor = in_[i].kc.merit();
    }
    SIPO_LAUNCHED("pdhg setup");

    const int check = hal ? std::max(1, o_.check_every) : o_.max_iters;
    const double itol = o_.infeas_tol > 0 ? o_.infeas_tol : 1e-6;
    if (hal) {
        // Warm-start multipliers that already form a Farkas ray (for instance those of a related
        // LP whose optimum shows the requested bound unreachable) certify infeasibility before
        // the first iteration: the candidate is max(lambda, 0) on the regions, put to the same
        // test as the iterates' rays.  Cold starts (all-zero multipliers) drop out of that test
        // after one reduction.  lut / llt hold zeros here and are rewritten by every iteration.
        std::vector<char> ok0;
        rc = farkas(L_.lu, L_.ll, kNoField, kNoField, itol, all, ok0);
        if (rc) return rc;
        std::vector<int> warm, rest;
        for (int i : all) (ok0[i] ? warm : rest).push_back(i);
        if (!warm.empty()) {
            for (int i : warm) {
                in_[i].status = SIPO_PRIMAL_INFEASIBLE;
                in_[i].cert = 2;
                in_[i].done = true;
                hin_[i].sel = 0;
            }
            set_flags(warm);
            rc = put_insts();
            if (rc) return rc;
            hipLaunchKernelGGL((k_certificate<T>), gV(), dim3(kThreads), 0, s_, F(L_.lu), F(L_.ll), (const T *)F(L_.lu),
                               (const T *)F(L_.ll), (const T *)nullptr, (const T *)nullptr,
                               (const uint8_t *)U8(L_.lab), insts(), segV());
            rc = set_active(rest);
            if (rc) return rc;
        }
        set_flags(rest);
        rc = put_insts();
        if (rc) return rc;
    }
    int it = 0, checks = 0;
    bool have_t = false;
    for (hipEvent_t &e : loop_ev_)
        if (!e) SIPO_HIP(hipEventCreate(&e));
    while (it < o_.max_iters && !active_.empty()) {
        const int nblk = std::min(check, o_.max_iters - it);
        rc = run_block(nblk);
        if (!rc) rc = flush_profile();
        if (rc) return rc;
        it += nblk;
        have_t = true;
        for (int i : active_) in_[i].iters = it;
        if (!hal) break;
        rc = get_scal();
        if (rc) return rc;
        std::vector<int> live;
        for (int i : active_) {
            const DevScal &h = hsc_[i];
            if (!std::isfinite(h.u) || !std::isfinite(h.v) || !std::isfinite(h.sum_l1) || !std::isfinite(h.sum_Ul2)) {
                in_[i].status = SIPO_NUMERICAL;
                in_[i].done = true;
            } else {
                live.push_back(i);
            }
        }
        // KKT of the PDHG output t; z_lambda(t) into tmp2
        rc = lambda_z(L_.lut, L_.llt, L_.tmp2, false);
        if (!rc) rc = kkt(L_.yt, L_.Dt, true, L_.lut, L_.llt, L_.tmp2, live);
        if (rc) return rc;
        ++checks;
        std::vector<int> open;
        for (int i : live) {
            const Kkt &k = in_[i].kc;
            if (!std::isfinite(k.r_p) || !std::isfinite(k.r_d)) { in_[i].status = SIPO_NUMERICAL; in_[i].done = true; }
            else if (k.rel() <= o_.tol) { in_[i].status = SIPO_OPTIMAL; in_[i].done = true; }
            else open.push_back(i);
        }
        // infeasibility: lambda(t) - lambda(z), then lambda(t) - lambda(t at the previous check)
        for (int i : open) in_[i].fk = INFINITY;
        std::vector<char> ok1, ok2;
        rc = farkas(L_.lut, L_.llt, L_.luo, L_.llo, itol, open, ok1);
        if (rc) return rc;
        std::vector<int> second;
        for (int i : open) {
            if (ok1[i]) { in_[i].status = SIPO_PRIMAL_INFEASIBLE; in_[i].cert = 0; in_[i].done = true; }
            else second.push_back(i);
        }
        rc = farkas(L_.lut, L_.llt, L_.snap_u, L_.snap_l, itol, second, ok2);
        if (rc) return rc;
        // then lambda(t) itself, and lambda(t) - lambda at the last restart: for an infeasible LP the
        // restarted iterates' multipliers grow along the ray, so their direction approaches it; the
        // multipliers of a feasible LP carry the objective's price and fail the scalar conditions
        std::vector<int> third, fourth, cont;
        for (int i : second) {
            if (ok2[i]) { in_[i].status = SIPO_PRIMAL_INFEASIBLE; in_[i].cert = 1; in_[i].done = true; }
            else third.push_back(i);
        }
        std::vector<char> ok3, ok4;
        rc = farkas(L_.lut, L_.llt, kNoField, kNoField, itol, third, ok3);
        if (rc) return rc;
        for (int i : third) {
            if (ok3[i]) { in_[i].status = SIPO_PRIMAL_INFEASIBLE; in_[i].cert = 3; in_[i].done = true; }
            else fourth.push_back(i);
        }
        rc = farkas(L_.lut, L_.llt, L_.lu0, L_.ll0, itol, fourth, ok4);
        if (rc) return rc;
        for (int i : fourth) {
            if (ok4[i]) { in_[i].status = SIPO_PRIMAL_INFEASIBLE; in_[i].cert = 4; in_[i].done = true; }
            else cont.push_back(i);
        }
        if (o_.progress_every > 0 && checks % o_.progress_every == 0)
            for (int i : live) {
                const Kkt &k = in_[i].kc;
                fprintf(stderr, "[sipo] instance %d: iteration %d, relative KKT %.3e (primal %.3e dual %.3e gap %.3e), "
                        "restarts %d, least Farkas violation %.2e\n", i, it, k.rel(), k.eps_p, k.eps_d, k.eps_gap,
                        in_[i].restarts, in_[i].fk);
            }
        set_flags(cont);
        rc = put_insts();
        if (rc) return rc;
        copyV(L_.snap_u, L_.lut, true);
        copyV(L_.snap_l, L_.llt, true);
        // restart rules on the l2 merit of the relative KKT residuals
        std::vector<int> rst;
        for (int i : cont) {
            Inst &I = in_[i];
            const double m = I.kc.merit();
            if (m <= 0.2 * I.m_anchor || (m <= 0.8 * I.m_anchor && m > I.m_prev) ||
                (double)(it - I.k_restart) >= 0.36 * (double)it)
                rst.push_back(i);
            else
                I.m_prev = m;
        }
        if (!rst.empty()) {
            // movement since the previous restart -> primal weight
            std::vector<double> dy2(B_), dlu2(B_), dll2(B_);
            hipLaunchKernelGGL((k_wdist<T>), gS(), dim3(kThreads), 0, s_, (const T *)F(L_.yt), (const T *)F(L_.ylast),
                               (const T *)F(L_.Tj), segS(), partials());
            rc = finish(false, rst, 1);
            if (rc) return rc;
            for (int i : rst) dy2[i] = sum(i, 0);
            hipLaunchKernelGGL((k_wdist<T>), gV(), dim3(kThreads), 0, s_, (const T *)F(L_.lut), (const T *)F(L_.lul),
                               (const T *)F(L_.s_up), segV(), partials());
            rc = finish(true, rst, 1);
            if (rc) return rc;
            for (int i : rst) dlu2[i] = sum(i, 0);
            hipLaunchKernelGGL((k_wdist<T>), gV(), dim3(kThreads), 0, s_, (const T *)F(L_.llt), (const T *)F(L_.lll),
                               (const T *)F(L_.s_lo), segV(), partials());
            rc = finish(true, rst, 1);
            if (rc) return rc;
            for (int i : rst) dll2[i] = sum(i, 0);
            // z, z0 and the restart point become t
            set_flags(rst);
            rc = put_insts();
            if (rc) return rc;
            for (size_t dst : {L_.y, L_.y0, L_.ylast}) copyS(dst, L_.yt, true);
            for (size_t dst : {L_.lu, L_.lu0, L_.lul}) copyV(dst, L_.lut, true);
            for (size_t dst : {L_.ll, L_.ll0, L_.lll}) copyV(dst, L_.llt, true);
            for (size_t dst : {L_.D, L_.D0}) copyV(dst, L_.Dt, true);
            rc = lambda_z(L_.lu, L_.ll, L_.z, true);
            if (!rc) rc = finish(true, rst, 2);
            if (rc) return rc;
            for (int i : rst) {
                Inst &I = in_[i];
                DevScal &h = hsc_[i];
                const double du = h.ut_done - I.last_u, dv = h.vt_done - I.last_v;
                const double dx = std::sqrt(dy2[i] + (I.Tu > 0 ? du * du / I.Tu : 0.0) + (I.Tv > 0 ? dv * dv / I.Tv : 0.0));
                const double dl = std::sqrt(dlu2[i] + dll2[i]);
                if (dx > 1e-10 && dl > 1e-10) I.omega = std::exp(0.5 * std::log(dl / dx) + 0.5 * std::log(I.omega));
                h.u = h.u0 = I.last_u = h.ut_done;
                h.v = h.v0 = I.last_v = h.vt_done;
                h.init_l1 = sum(i, 0);
                h.init_Ul2 = sum(i, 1);
                h.tau_fac = eta / I.omega;
                h.sig_fac = eta * I.omega;
                h.tau_u = eta * I.Tu / I.omega;
                h.tau_v = eta * I.Tv / I.omega;
                I.m_anchor = I.kc.merit();
                I.m_prev = 1e300;
                I.k_restart = it;
                ++I.restarts;
            }
            rc = put_scal();   // restarting instances take the host values; the others keep theirs
            if (rc) return rc;
            hipLaunchKernelGGL(k_scalars_init, dim3(1), dim3(kThreads), 0, s_, scal(), insts(), B_);
        }
        if (cont.size() != active_.size()) {
            rc = set_active(cont);
            if (rc) return rc;
        }
    }
    if (loop_started_) SIPO_HIP(hipEventRecord(loop_ev_[1], s_));
    // ---------------- returned points: the PDHG output t (restarted) or z = t (plain)
    rc = get_scal();
    if (!rc) rc = set_active(all);
    if (rc) return rc;
    std::vector<int> from_t, certs, recheck;
    for (int i = 0; i < B_; ++i) {
        if (hal && have_t && in_[i].cert != 2) {
            from_t.push_back(i);
            if (in_[i].status == SIPO_PRIMAL_INFEASIBLE) certs.push_back(i);
        }
        if (in_[i].status == SIPO_ITER_LIMIT || in_[i].status == SIPO_NUMERICAL || !hal) recheck.push_back(i);
    }
    std::vector<double> ru(B_), rv(B_);
    for (int i = 0; i < B_; ++i) {
        const bool t = hal && have_t && in_[i].cert != 2;
        ru[i] = t ? hsc_[i].ut_done : hsc_[i].u;
        rv[i] = t ? hsc_[i].vt_done : hsc_[i].v;
    }
    if (!from_t.empty()) {
        set_flags(from_t);
        rc = put_insts();
        if (rc) return rc;
        copyS(L_.y, L_.yt, true);
        copyV(L_.D, L_.Dt, true);
        std::vector<int> plain_copy;
        for (int i : from_t)
            if (in_[i].status != SIPO_PRIMAL_INFEASIBLE) plain_copy.push_back(i);
        set_flags(plain_copy);
        rc = put_insts();
        if (rc) return rc;
        copyV(L_.lu, L_.lut, true);
        copyV(L_.ll, L_.llt, true);
        // certificates: max(lambda(t) - b, 0) with b the pre-step (0), snapshot (1), zero (3) or
        // restart point (4) multipliers of the test that accepted it
        const struct { int cert; size_t bu, bl; } kinds[] = {
            {0, L_.luo, L_.llo}, {1, L_.snap_u, L_.snap_l}, {3, kNoField, kNoField}, {4, L_.lu0, L_.ll0}};
        for (const auto &kd : kinds) {
            std::vector<int> sel;
            for (int i : certs)
                if (in_[i].cert == kd.cert) sel.push_back(i);
            if (sel.empty()) continue;
            set_flags(sel);
            rc = put_insts();
            if (rc) return rc;
            hipLaunchKernelGGL((k_certificate<T>), gV(), dim3(kThreads), 0, s_, F(L_.lu), F(L_.ll), (const T *)F(L_.lut),
                               (const T *)F(L_.llt), Fz(kd.bu), Fz(kd.bl), (const uint8_t *)U8(L_.lab), insts(),
                               segV());
        }
    }
    if (!recheck.empty()) {
        // KKT of the returned point (its u, v passed as the "t" scalars)
        for (int i : recheck) { hsc_[i].ut_done = ru[i]; hsc_[i].vt_done = rv[i]; }
        rc = set_active(recheck);
        if (!rc) rc = lambda_z(L_.lu, L_.ll, L_.z, false);
        if (!rc) rc = kkt(L_.y, L_.D, true, L_.lu, L_.ll, L_.z, recheck);
        if (rc) return rc;
        rc = set_active(all);
        if (rc) return rc;
    }
    if (mask_) {
        // a requested dose is returned on the whole volume (the masked operators and the dual step kept
        // it on the LP's rows only)
        bool full = false;
        for (int i = 0; i < B_; ++i) full = full || probs_[i].dose_out;
        mask_ = false;
        if (full) {
            rc = dose(L_.y, L_.D);
            if (rc) return rc;
        }
    }
    rc = unpack();
    if (rc) return rc;
    SIPO_LAUNCHED("pdhg finish");
    SIPO_HIP(hipStreamSynchronize(s_));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    float loop_ms = 0.f;
    if (loop_started_) SIPO_HIP(hipEventElapsedTime(&loop_ms, loop_ev_[0], loop_ev_[1]));
    for (int i = 0; i < B_; ++i) {
        const Inst &I = in_[i];
        sipo_pdhg_result &r = res[i];
        r.status = I.status;
        r.iters = I.iters;
        r.restarts = I.restarts;
        r.primal_obj = I.kc.p;
        r.dual_obj = I.kc.d;
        r.rel_primal = I.kc.eps_p;
        r.rel_dual = I.kc.eps_d;
        r.rel_gap = I.kc.eps_gap;
        r.u = ru[i];
        r.v = rv[i];
        r.tau = I.tau;
        r.sigma = I.sigma;
        r.omega = I.omega;
        r.time_ms = ms;
        r.loop_ms = loop_ms;
        for (int ph = 0; ph < SIPO_NUM_PHASES; ++ph) {
            r.phase_ms[ph] = phase_ms_[ph];
            r.phase_launches[ph] = phase_n_[ph];
        }
        for (int k = 0; k < 8; ++k) r.op_config[k] = 0;
        r.tiles_2d[0] = b2d_ ? t2d_.bx : 0;
        r.tiles_2d[1] = b2d_ ? t2d_.vb : 0;
        r.tiles_2d[2] = b2d_ ? t2d_.fb : 0;
        if (masked_run_ && I.t3) {
            r.op_config[0] = I.p->p3d_zc;
            r.op_config[1] = I.p->bp3d_zc;
            r.op_config[2] = bsp_[i].parts;
            r.op_config[3] = I.p->has_psf ? I.p->blur_zc : 0;
            const bool queued = !pqueue_.empty() && pqueue_[i] > 0 && steps_[i] && psp_[i].parts == 1;
            r.op_config[4] = queued ? pqueue_[i] : -1;
            r.op_config[5] = fused_[i] ? 1 : -1;
            r.op_config[6] = I.p->p3d_skip ? 1 : -1;
            r.op_config[7] = steps_[i] ? p3d_list_chunk(I.p, step_list(i, false)) : 0;
        }
    }
    return SIPO_OK;
}

static int validate(const sipo_problem &pb, const sipo_pdhg_options &o, int idx, sipo_dtype dt) {
    int rc = check_plan(pb.plan);
    if (rc) return rc;
    SIPO_REQUIRE(pb.plan->dtype == dt, "problem %d: plan precision differs from problem 0", idx);
    SIPO_REQUIRE(pb.labels && pb.act && pb.y && pb.lam_up && pb.lam_lo, "problem %d: a required pointer is NULL", idx);
    SIPO_REQUIRE(pb.u_free == 0 || pb.u_free == 1, "problem %d: u_free must be 0 or 1", idx);
    SIPO_REQUIRE(pb.v_free == 0 || pb.v_free == 1, "problem %d: v_free must be 0 or 1", idx);
    SIPO_REQUIRE(std::isfinite(pb.w1) && std::isfinite(pb.w2) && pb.w1 >= 0 && pb.w2 >= 0,
                 "problem %d: weights must be finite and >= 0", idx);
    SIPO_REQUIRE(std::isfinite(pb.band_cap) && std::isfinite(pb.lo_scalar) && std::isfinite(pb.hi_scalar),
                 "problem %d: scalars must be finite", idx);
    SIPO_REQUIRE(o.mode == SIPO_PDHG_PLAIN || o.mode == SIPO_PDHG_RESTARTED, "unknown PDHG mode %d", o.mode);
    SIPO_REQUIRE(o.max_iters >= 1, "max_iters must be >= 1");
    SIPO_REQUIRE(!(o.profile && o.use_graph), "profile and use_graph cannot be combined");
    SIPO_REQUIRE(o.mode == SIPO_PDHG_PLAIN || o.check_every >= 1, "check_every must be >= 1");
    SIPO_REQUIRE(!(o.eta >= 1.0), "eta must be < 1");
    SIPO_REQUIRE(std::isfinite(o.scalar_weight) && o.scalar_weight >= 0, "scalar_weight must be finite and >= 0");
    SIPO_REQUIRE(o.progress_every >= 0, "progress_every must be >= 0");
    SIPO_REQUIRE(o.tune_operators == 0 || o.tune_operators == 1, "tune_operators must be 0 or 1");
    {
        const int *c = o.op_config;
        SIPO_REQUIRE(c[0] == 0 || c[0] == 8 || c[0] == 16 || c[0] == 32, "op_config[0] (projector slices per thread) "
                     "must be 0, 8, 16 or 32, not %d", c[0]);
        SIPO_REQUIRE(c[1] == 0 || c[1] == 4 || c[1] == 8 || c[1] == 16, "op_config[1] (backprojector slices per thread) "
                     "must be 0, 4, 8 or 16, not %d", c[1]);
        SIPO_REQUIRE(c[2] >= 0 && c[2] <= kMaxSplitB, "op_config[2] (backprojector view splits) must be in [0, %d], not %d",
                     kMaxSplitB, c[2]);
        SIPO_REQUIRE(c[3] == 0 || c[3] == 4 || c[3] == 8 || c[3] == 16, "op_config[3] (blur slices per chunk) must be "
                     "0, 4, 8 or 16, not %d", c[3]);
        SIPO_REQUIRE(c[4] >= -1 && c[4] <= 16, "op_config[4] (projector work queue) must be in [-1, 16], not %d", c[4]);
        SIPO_REQUIRE(c[5] >= -1 && c[5] <= 1, "op_config[5] (primal step) must be -1, 0 or 1, not %d", c[5]);
        SIPO_REQUIRE(c[6] >= -1 && c[6] <= 1, "op_config[6] (candidate skipping) must be -1, 0 or 1, not %d", c[6]);
        SIPO_REQUIRE(c[7] >= 0 && c[7] <= 2, "op_config[7] (listed steps per staged chunk) must be 0, 1 or 2, not %d",
                     c[7]);
        const int *t = o.tiles_2d;
        SIPO_REQUIRE(t[0] == 0 || t[0] == 16 || t[0] == 32 || t[0] == 64, "tiles_2d[0] (backprojector tile width) must "
                     "be 0, 16, 32 or 64, not %d", t[0]);
        SIPO_REQUIRE(t[1] == 0 || t[1] == 8 || t[1] == 16 || t[1] == 32, "tiles_2d[1] (views per staged batch) must be "
                     "0, 8, 16 or 32, not %d", t[1]);
        SIPO_REQUIRE(t[2] == 0 || t[2] == 32 || t[2] == 64 || t[2] == 128, "tiles_2d[2] (projector bins per bundle) "
                     "must be 0, 32, 64 or 128, not %d", t[2]);
    }
    return SIPO_OK;
}

}  // namespace sipo

using namespace sipo;

extern "C" {

size_t sipo_pdhg_workspace_size(const sipo_problem *probs, int32_t n, const sipo_pdhg_options *) {
    if (!probs || n < 1 || n > 65536) return 0;
    for (int i = 0; i < n; ++i)
        if (!probs[i].plan) return 0;
    return make_layout(probs, n).total;
}

int sipo_pdhg_solve(const sipo_problem *probs, int32_t n, const sipo_pdhg_options *opts, void *workspace,
                    size_t ws_bytes, sipo_pdhg_result *results, void *stream) {
    SIPO_REQUIRE(probs && opts && results && n >= 1 && n <= 65536, "NULL argument or n outside [1, 65536]");
    SIPO_REQUIRE(probs[0].plan != nullptr, "problem 0: plan is NULL");
    const sipo_dtype dt = probs[0].plan->dtype;
    for (int i = 0; i < n; ++i) {
        SIPO_REQUIRE(probs[i].plan != nullptr, "problem %d: plan is NULL", i);
        int rc = validate(probs[i], *opts, i, dt);
        if (rc) return rc;
    }
    const Layout L = make_layout(probs, n);
    SIPO_REQUIRE(workspace != nullptr, "workspace is NULL");
    if (ws_bytes < L.total) return fail(SIPO_E_WORKSPACE, "workspace of %zu bytes < %zu required", ws_bytes, L.total);
    hipStream_t s = (hipStream_t)stream;
    SIPO_REQUIRE(!(opts->use_graph && s == nullptr), "graph capture needs a non-default stream");
    return dt == SIPO_F64 ? Solver<double>(probs, n, *opts, (char *)workspace, L, s).run(results)
                          : Solver<float>(probs, n, *opts, (char *)workspace, L, s).run(results);
}

}  // extern "C"
