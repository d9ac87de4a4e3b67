// Matrix-free PDHG for the unified Charnes-Cooper LP (Sec. 2.8, Supp. 6.1).
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
// All iteration-varying scalars live in a device block, so an iteration is a
// fixed sequence of launches with fixed arguments; a block of iterations can
// be captured once in a HIP graph and replayed.  Reductions are two-level
// (per-block FP64 partials summed in a fixed order by one block), so results
// are deterministic.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

#include "sipo_internal.hpp"

namespace sipo {

constexpr int kRedBlocks = 1024;   // upper bound on reduction blocks
constexpr int kNS = 8;             // sums carried per reduction
constexpr int kThreads = 256;

// Device scalar block (FP64): everything that changes from one iteration to the next.
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
    double sums[kNS];         // last generic reduction result
};

struct LPConst {
    int u_free, v_free;
    double w1, w2, h;         // weights and band cap
    double lo_s, hi_s;        // scalar bounds when arrays are absent
};

// -------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

template <int NS>
__device__ __forceinline__ void block_sums(double (&v)[NS], double *partials) {
    __shared__ double red[kThreads / 64][NS];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const double s = wave_sum(v[k]);
        if (lane == 0) red[w][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < NS) {
        double s = 0.0;
        for (int i = 0; i < kThreads / 64; ++i) s += red[i][threadIdx.x];
        partials[blockIdx.x * kNS + threadIdx.x] = s;
    }
}

// Total of column k of the per-block partials, by one block of kThreads threads:
// strided per-thread sums, then a fixed tree, so the result does not depend on timing.
template <bool MAX>
__device__ double block_total(const double *__restrict__ partials, int nblocks, int k, double *sh) {
    double a = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kThreads) {
        const double v = partials[b * kNS + k];
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

// Sum per-block partials into dst[0..ns).
__global__ void __launch_bounds__(kThreads) finish_sums(const double *__restrict__ partials, int nblocks,
                                                         double *dst, int ns) {
    __shared__ double sh[kThreads];
    for (int k = 0; k < ns; ++k) {
        const double r = block_total<false>(partials, nblocks, k, sh);
        if (threadIdx.x == 0) dst[k] = r;
    }
}

#define GRID_LOOP(i, n) \
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < (n); i += (size_t)gridDim.x * blockDim.x)

template <typename T>
__device__ __forceinline__ T ld_or(const T *p, size_t i, double s) { return p ? p[i] : (T)s; }

// ------------------------------------------------------------- setup kernels
// y <- act ? max(y, 0) : 0  (warm start projected onto X)
template <typename T>
__global__ void k_project_y(T *y, const uint8_t *act, size_t n) {
    GRID_LOOP(i, n) y[i] = act[i] ? (y[i] > (T)0 ? y[i] : (T)0) : (T)0;
}

// lambda projected onto its regions and >= 0; z = lambda_up - lambda_lo; [0] sum_band lambda1, [1] sum_gel U lambda2.
template <typename T>
__global__ void k_lambda_z(T *lu, T *ll, T *z, const uint8_t *lab, const T *hi, LPConst c, size_t n,
                           double *partials) {
    double acc[kNS] = {0, 0, 0, 0, 0, 0, 0, 0};
    GRID_LOOP(i, n) {
        const uint8_t L = lab[i];
        T a = L ? (lu[i] > (T)0 ? lu[i] : (T)0) : (T)0;
        T b = (L == 2) ? (ll[i] > (T)0 ? ll[i] : (T)0) : (T)0;
        lu[i] = a;
        ll[i] = b;
        z[i] = a - b;
        if (L == 1) acc[0] += (double)a;
        if (L == 2) acc[1] += (double)ld_or(hi, i, c.hi_s) * (double)a;
    }
    block_sums<kNS>(acc, partials);
}

// w = 1 on band, 2 on gel (absolute column weights of G)
template <typename T>
__global__ void k_colweight(T *w, const uint8_t *lab, size_t n) {
    GRID_LOOP(i, n) w[i] = lab[i] == 1 ? (T)1 : (lab[i] == 2 ? (T)2 : (T)0);
}

template <typename T>
__global__ void k_act_to_float(T *a, const uint8_t *act, size_t n) {
    GRID_LOOP(i, n) a[i] = act[i] ? (T)1 : (T)0;
}

// T_j = act & colsum > 0 ? 1 / colsum : 0
template <typename T>
__global__ void k_inv_colsum(T *t, const uint8_t *act, size_t n) {
    GRID_LOOP(i, n) t[i] = (act[i] && t[i] > (T)0) ? (T)1 / t[i] : (T)0;
}

// S_up = 1/(R + [band, u free] + [gel, v free] U), S_lo = [gel] 1/R;
// [0] |band|, [1] sum_gel U, [2] ||h||^2, [3] |gel|
template <typename T>
__global__ void k_row_scaling(const T *R, T *s_up, T *s_lo, const uint8_t *lab, const T *lo, const T *hi, LPConst c,
                              size_t n, double *partials) {
    double acc[kNS] = {0, 0, 0, 0, 0, 0, 0, 0};
    GRID_LOOP(i, n) {
        const uint8_t L = lab[i];
        const T r = R[i];
        T su = 0, sl = 0;
        if (L == 1) {
            const T rs = r + (c.u_free ? (T)1 : (T)0);
            su = rs > (T)0 ? (T)1 / rs : (T)0;
            acc[0] += 1.0;
            if (!c.u_free) acc[2] += c.h * c.h;
        } else if (L == 2) {
            const double U = (double)ld_or(hi, i, c.hi_s), Lo = (double)ld_or(lo, i, c.lo_s);
            const T rs = r + (c.v_free ? (T)U : (T)0);
            su = rs > (T)0 ? (T)1 / rs : (T)0;
            sl = r > (T)0 ? (T)1 / r : (T)0;
            acc[1] += U;
            acc[2] += Lo * Lo + (c.v_free ? 0.0 : U * U);
            acc[3] += 1.0;
        }
        s_up[i] = su;
        s_lo[i] = sl;
    }
    block_sums<kNS>(acc, partials);
}

// --------------------------------------------------------- iteration kernels
// t.y = act ? max(0, y - tau q) : 0 with tau = tau_fac T_j (or tau_fac); y <- w ((1+rho) t.y - rho y) + (1-w) y0.
template <typename T>
__global__ void k_primal(T *__restrict__ y, T *__restrict__ yt, const T *__restrict__ q, const T *__restrict__ Tj,
                         const uint8_t *__restrict__ act, const T *__restrict__ y0, const DevScal *__restrict__ sc,
                         size_t n) {
    const T tf = (T)sc->tau_fac;
    const T w = (T)sc->w, rho = (T)sc->rho;
    GRID_LOOP(i, n) {
        T t = (T)0;
        const T yo = y[i];
        if (act[i]) {
            const T st = Tj ? tf * Tj[i] : tf;
            t = yo - st * q[i];
            t = t > (T)0 ? t : (T)0;
        }
        yt[i] = t;
        y[i] = y0 ? w * (((T)1 + rho) * t - rho * yo) + ((T)1 - w) * y0[i] : t;
    }
}

// Dual step on voxels from D_t (= K P^T t.y) and D (= K P^T z.y); Halpern update of lambda and D;
// z_lambda for the next step; on check iterations t.lambda and the pre-step lambda are kept.
// [0] sum_band lambda1, [1] sum_gel U lambda2 of the new lambda.
template <typename T>
__global__ void k_dual(const T *__restrict__ Dt, T *__restrict__ D, const T *__restrict__ D0, T *__restrict__ lu,
                       T *__restrict__ ll, const T *__restrict__ lu0, const T *__restrict__ ll0, T *__restrict__ z,
                       const uint8_t *__restrict__ lab, const T *__restrict__ lo, const T *__restrict__ hi,
                       const T *__restrict__ s_up, const T *__restrict__ s_lo, T *__restrict__ lut,
                       T *__restrict__ llt, T *__restrict__ luo, T *__restrict__ llo, const DevScal *__restrict__ sc,
                       LPConst c, size_t n, double *partials) {
    const double sf = sc->sig_fac;
    const T ub = (T)(c.u_free ? sc->ubar : c.h);
    const T vb = (T)(c.v_free ? sc->vbar : 1.0);
    const T w = (T)sc->w, rho = (T)sc->rho, w1 = (T)1 - w, rp = (T)1 + rho;
    double acc[kNS] = {0, 0, 0, 0, 0, 0, 0, 0};
    GRID_LOOP(i, n) {
        const T dt = Dt[i], dz = D[i];
        D[i] = D0 ? w * (rp * dt - rho * dz) + w1 * D0[i] : dt;
        const uint8_t L = lab[i];
        if (L == 0) continue;
        const T Db = (T)2 * dt - dz;
        const T su = s_up ? (T)sf * s_up[i] : (T)sf;
        const T a_old = lu[i];
        T a = a_old + su * (Db - (L == 1 ? ub : vb * ld_or(hi, i, c.hi_s)));
        a = a > (T)0 ? a : (T)0;
        const T a_new = lu0 ? w * (rp * a - rho * a_old) + w1 * lu0[i] : a;
        lu[i] = a_new;
        if (lut) { lut[i] = a; luo[i] = a_old; }
        T zz = a_new;
        if (L == 1) {
            acc[0] += (double)a_new;
        } else {
            const T sl = s_lo ? (T)sf * s_lo[i] : (T)sf;
            const T b_old = ll[i];
            T b = b_old + sl * (ld_or(lo, i, c.lo_s) - Db);
            b = b > (T)0 ? b : (T)0;
            const T b_new = ll0 ? w * (rp * b - rho * b_old) + w1 * ll0[i] : b;
            ll[i] = b_new;
            if (llt) { llt[i] = b; llo[i] = b_old; }
            zz = a_new - b_new;
            acc[1] += (double)ld_or(hi, i, c.hi_s) * (double)a_new;
        }
        z[i] = zz;
    }
    block_sums<kNS>(acc, partials);
}

// Next scalar primal step from the current z and the lambda sums.
__device__ __forceinline__ void roll_next(DevScal *sc, const LPConst &c) {
    sc->ut = c.u_free ? fmax(0.0, sc->u - sc->tau_u * (c.w1 - sc->sum_l1)) : c.h;
    sc->vt = c.v_free ? fmax(0.0, sc->v - sc->tau_v * (c.w2 - sc->sum_Ul2)) : 1.0;
    sc->ubar = 2.0 * sc->ut - sc->u;
    sc->vbar = 2.0 * sc->vt - sc->v;
}

// One block: finish the lambda sums, apply the Halpern update to (u, v), prepare the next step.
__global__ void __launch_bounds__(kThreads) k_scalars(const double *__restrict__ partials, int nblocks,
                                                       DevScal *sc, LPConst c) {
    __shared__ double sh[kThreads];
    const double s0 = block_total<false>(partials, nblocks, 0, sh);
    const double s1 = block_total<false>(partials, nblocks, 1, sh);
    if (threadIdx.x != 0) return;
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

// After a (re)start: sums of lambda in sums[0..1]; set the weight and the first step.
__global__ void k_scalars_init(DevScal *sc, LPConst c) {
    sc->sum_l1 = sc->sums[0];
    sc->sum_Ul2 = sc->sums[1];
    sc->k_in = 0.0;
    sc->w = sc->halpern != 0.0 ? 0.5 : 1.0;
    roll_next(sc, c);
}

// ---------------------------------------------------------------- KKT pieces
// Voxel side at (D, u, v, lambda): [0] ||(Gx-h)^+||^2 voxel rows, [1] sum L lambda3,
// [2] sum_band lambda1, [3] sum_gel U lambda2.
template <typename T>
__global__ void k_kkt_vox(const T *D, const T *lu, const T *ll, const uint8_t *lab, const T *lo, const T *hi,
                          LPConst c, double u, double v, size_t n, double *partials) {
    double acc[kNS] = {0, 0, 0, 0, 0, 0, 0, 0};
    GRID_LOOP(i, n) {
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
    block_sums<kNS>(acc, partials);
}

// Ray side: [0] sum_act min(q,0)^2, [1] sum_act y^-^2 + sum_mask y^2.
template <typename T>
__global__ void k_kkt_ray(const T *q, const T *y, const uint8_t *act, size_t n, double *partials) {
    double acc[kNS] = {0, 0, 0, 0, 0, 0, 0, 0};
    GRID_LOOP(i, n) {
        const double yi = (double)y[i];
        if (act[i]) {
            const double qi = (double)q[i];
            if (qi < 0) acc[0] += qi * qi;
            if (yi < 0) acc[1] += yi * yi;
        } else {
            acc[1] += yi * yi;
        }
    }
    block_sums<kNS>(acc, partials);
}

// Farkas candidate d = max(a - b, 0) on the regions -> z_d; [0] sum L d3, [1] sum_band d1,
// [2] sum_gel U d2, [3] ||d||_1.
template <typename T>
__global__ void k_ray_candidate(const T *alu, const T *all, const T *blu, const T *bll, T *zd, const uint8_t *lab,
                                const T *lo, const T *hi, LPConst c, size_t n, double *partials) {
    double acc[kNS] = {0, 0, 0, 0, 0, 0, 0, 0};
    GRID_LOOP(i, n) {
        const uint8_t L = lab[i];
        T zz = 0;
        if (L) {
            T a = alu[i] - blu[i];
            a = a > (T)0 ? a : (T)0;
            zz = a;
            acc[3] += (double)a;
            if (L == 1) {
                acc[1] += (double)a;
            } else {
                T b = all[i] - bll[i];
                b = b > (T)0 ? b : (T)0;
                zz = a - b;
                acc[0] += (double)ld_or(lo, i, c.lo_s) * (double)b;
                acc[2] += (double)ld_or(hi, i, c.hi_s) * (double)a;
                acc[3] += (double)b;
            }
        }
        zd[i] = zz;
    }
    block_sums<kNS>(acc, partials);
}

// Certificate output: out = max(a - b, 0) on the regions (lambda_lo on gel only).
template <typename T>
__global__ void k_certificate(T *olu, T *oll, const T *alu, const T *all, const T *blu, const T *bll,
                              const uint8_t *lab, size_t n) {
    GRID_LOOP(i, n) {
        const uint8_t L = lab[i];
        T a = L ? alu[i] - blu[i] : (T)0;
        T b = (L == 2) ? all[i] - bll[i] : (T)0;
        olu[i] = a > (T)0 ? a : (T)0;
        oll[i] = b > (T)0 ? b : (T)0;
    }
}

// [0] max over act of -q (clipped at 0), [1] max over act of |q|
template <typename T>
__global__ void k_ray_check(const T *q, const uint8_t *act, size_t n, double *partials) {
    __shared__ double m0[kThreads], m1[kThreads];
    double a0 = 0.0, a1 = 0.0;
    GRID_LOOP(i, n) {
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

__global__ void __launch_bounds__(kThreads) finish_max(const double *__restrict__ partials, int nblocks,
                                                        double *dst) {
    __shared__ double sh[kThreads];
    const double m0 = block_total<true>(partials, nblocks, 0, sh);
    const double m1 = block_total<true>(partials, nblocks, 1, sh);
    if (threadIdx.x == 0) { dst[0] = m0; dst[1] = m1; }
}

// power iteration: G^T-side combination of the rows of G x with D = K P^T y,
// [0] sum_band (D - u), [1] sum_gel U (D - v U)
template <typename T>
__global__ void k_pi_rows(const T *D, T *z, const uint8_t *lab, const T *hi, LPConst c, double u, double v, size_t n,
                          double *partials) {
    double acc[kNS] = {0, 0, 0, 0, 0, 0, 0, 0};
    GRID_LOOP(i, n) {
        const uint8_t L = lab[i];
        T zz = 0;
        if (L == 1) {
            const double r = (double)D[i] - (c.u_free ? u : 0.0);
            zz = (T)r;
            acc[0] += r;
        } else if (L == 2) {
            const double U = (double)ld_or(hi, i, c.hi_s);
            const double r = (double)D[i] - (c.v_free ? v * U : 0.0);
            zz = (T)(r + (double)D[i]);   // gel-up row minus gel-lo row (-D)
            acc[1] += U * r;
        }
        z[i] = zz;
    }
    block_sums<kNS>(acc, partials);
}

// y <- act ? q : 0 ; [0] sum y^2
template <typename T>
__global__ void k_pi_mask(T *y, const T *q, const uint8_t *act, size_t n, double *partials) {
    double acc[kNS] = {0, 0, 0, 0, 0, 0, 0, 0};
    GRID_LOOP(i, n) {
        const T v = act[i] ? q[i] : (T)0;
        y[i] = v;
        acc[0] += (double)v * (double)v;
    }
    block_sums<kNS>(acc, partials);
}

template <typename T>
__global__ void k_scale(T *a, double s, size_t n) {
    GRID_LOOP(i, n) a[i] = (T)((double)a[i] * s);
}

template <typename T>
__global__ void k_copy(T *dst, const T *src, size_t n) {
    GRID_LOOP(i, n) dst[i] = src[i];
}

// weighted movement: [0] sum (a-b)^2 / w over w > 0
template <typename T>
__global__ void k_wdist(const T *a, const T *b, const T *w, size_t n, double *partials) {
    double acc[kNS] = {0, 0, 0, 0, 0, 0, 0, 0};
    GRID_LOOP(i, n) {
        const double wi = (double)w[i];
        if (wi > 0) {
            const double d = (double)a[i] - (double)b[i];
            acc[0] += d * d / wi;
        }
    }
    block_sums<kNS>(acc, partials);
}

// ================================================================= host side
struct Workspace {
    // sinogram-sized, internal layout
    void *q, *Tj, *yt, *y0, *ylast, *y_int;
    uint8_t *act_int;
    // volume-sized
    void *D, *Dt, *D0, *z, *tmp, *tmp2, *s_up, *s_lo, *lut, *llt, *luo, *llo, *snap_u, *snap_l, *lu0, *ll0,
        *lul, *lll, *vol_t;
    double *partials;
    DevScal *scal;
};

static size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

static size_t layout(const sipo_problem &pb, Workspace *ws, char *base) {
    const sipo_plan p = pb.plan;
    const size_t eb = p->elem_bytes();
    const size_t sb = align_up(p->sino_elems() * eb), vb = align_up(p->vol_elems() * eb);
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        void *r = base ? (void *)(base + off) : nullptr;
        off += bytes;
        return r;
    };
    Workspace w{};
    w.q = take(sb); w.Tj = take(sb); w.yt = take(sb); w.y0 = take(sb); w.ylast = take(sb);
    const bool t3 = p->fast3d();
    w.y_int = t3 ? take(sb) : nullptr;
    w.act_int = t3 ? (uint8_t *)take(align_up(p->sino_elems())) : nullptr;
    w.vol_t = t3 ? take(vb) : nullptr;
    w.D = take(vb); w.Dt = take(vb); w.D0 = take(vb); w.z = take(vb); w.tmp = take(vb); w.tmp2 = take(vb);
    w.s_up = take(vb); w.s_lo = take(vb); w.lut = take(vb); w.llt = take(vb); w.luo = take(vb); w.llo = take(vb);
    w.snap_u = take(vb); w.snap_l = take(vb); w.lu0 = take(vb); w.ll0 = take(vb); w.lul = take(vb); w.lll = take(vb);
    w.partials = (double *)take(align_up(sizeof(double) * kRedBlocks * kNS));
    w.scal = (DevScal *)take(align_up(sizeof(DevScal)));
    if (ws) *ws = w;
    return off;
}

template <typename T>
class Solver {
  public:
    Solver(const sipo_problem &pb, const sipo_pdhg_options &o, const Workspace &w, hipStream_t s)
        : pb_(pb), o_(o), w_(w), s_(s), p_(pb.plan) {
        nv_ = p_->vol_elems();
        ns_ = p_->sino_elems();
        c_.u_free = pb.u_free;
        c_.v_free = pb.v_free;
        c_.w1 = pb.w1;
        c_.w2 = pb.w2;
        c_.h = pb.band_cap;
        c_.lo_s = pb.lo_scalar;
        c_.hi_s = pb.hi_scalar;
        lab_ = pb.labels;
        t3_ = p_->fast3d();
        act_ = t3_ ? w.act_int : pb.act;
        lo_ = (const T *)pb.lo;
        hi_ = (const T *)pb.hi;
        y_ = t3_ ? (T *)w.y_int : (T *)pb.y;
        lu_ = (T *)pb.lam_up;
        ll_ = (T *)pb.lam_lo;
        gv_ = std::max(1, (int)std::min<size_t>((nv_ + kThreads * 4 - 1) / (kThreads * 4), kRedBlocks));
        gs_ = std::max(1, (int)std::min<size_t>((ns_ + kThreads * 4 - 1) / (kThreads * 4), kRedBlocks));
    }
    ~Solver() {
        if (graph_exec_) (void)hipGraphExecDestroy(graph_exec_);
        for (hipEvent_t e : ev_) (void)hipEventDestroy(e);
    }

    int run(sipo_pdhg_result *res);

  private:
    const sipo_problem &pb_;
    sipo_pdhg_options o_;
    Workspace w_;
    hipStream_t s_;
    sipo_plan p_;
    size_t nv_, ns_;
    int gv_, gs_;
    LPConst c_;
    const uint8_t *lab_, *act_;
    bool t3_ = false;     // sinograms held in the internal [view][bin][z] layout
    const T *lo_, *hi_;
    T *y_, *lu_, *ll_;
    double h_norm_ = 0, c_norm_ = 0;
    double Tu_ = 0, Tv_ = 0;
    DevScal hs_{};
    hipGraphExec_t graph_exec_ = nullptr;
    int graph_len_ = 0;

    template <typename U>
    void copy(U *dst, const U *src, size_t n, int grid) {
        hipLaunchKernelGGL((k_copy<U>), dim3(grid), dim3(kThreads), 0, s_, dst, src, n);
    }
    T *V(void *p) { return (T *)p; }
    // operators on the solver's layouts: sinograms as held internally, volumes [z][y][x]
    int dose(const T *y, T *out) {   // out = K P^T y  (uses tmp when K != I)
        if (!p_->has_psf) {
            int rc = launch_backproject_t(p_, y, out, 0, s_);
            return rc ? rc : mark(SIPO_PHASE_BACKPROJECT);
        }
        int rc = launch_backproject_t(p_, y, w_.tmp, 0, s_);
        if (!rc) rc = mark(SIPO_PHASE_BACKPROJECT);
        if (!rc) rc = launch_blur(p_, w_.tmp, out, s_);
        return rc ? rc : mark(SIPO_PHASE_BLUR);
    }
    int adjoint(const T *z, T *out) {   // out = P K z
        const void *src = z;
        if (p_->has_psf) {
            int rc = launch_blur(p_, z, w_.tmp, s_);
            if (!rc) rc = mark(SIPO_PHASE_BLUR);
            if (rc) return rc;
            src = w_.tmp;
        }
        if (!t3_) {
            int rc = launch_project_t(p_, src, out, s_);
            return rc ? rc : mark(SIPO_PHASE_PROJECT);
        }
        int rc = launch_vol_to_t(p_, src, w_.vol_t, s_);
        if (!rc) rc = mark(SIPO_PHASE_TRANSPOSE);
        if (!rc) rc = launch_project_t(p_, w_.vol_t, out, s_);
        return rc ? rc : mark(SIPO_PHASE_PROJECT);
    }
    // ---- profile mode: a timeline of events between consecutive iteration launches
    bool prof_on_ = false;                // inside an iteration of a profiled solve
    std::vector<hipEvent_t> ev_;
    std::vector<int> ev_phase_;           // phase of the launch that ends at ev_[i]
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
    int flush_profile() {   // fold the recorded intervals into the phase totals
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
    int sums(int nblocks, int ns, double *host) {
        hipLaunchKernelGGL(finish_sums, dim3(1), dim3(kThreads), 0, s_, w_.partials, nblocks, w_.scal->sums, ns);
        SIPO_HIP(hipMemcpyAsync(host, w_.scal->sums, sizeof(double) * ns, hipMemcpyDeviceToHost, s_));
        SIPO_HIP(hipStreamSynchronize(s_));
        return SIPO_OK;
    }
    int get_scal() {
        SIPO_HIP(hipMemcpyAsync(&hs_, w_.scal, sizeof(DevScal), hipMemcpyDeviceToHost, s_));
        SIPO_HIP(hipStreamSynchronize(s_));
        return SIPO_OK;
    }
    int put_scal() {
        SIPO_HIP(hipMemcpyAsync(w_.scal, &hs_, sizeof(DevScal), hipMemcpyHostToDevice, s_));
        return SIPO_OK;
    }
    int lambda_z(T *lu, T *ll, T *z, double *sum_l1, double *sum_ul2) {
        hipLaunchKernelGGL((k_lambda_z<T>), dim3(gv_), dim3(kThreads), 0, s_, lu, ll, z, lab_, hi_, c_, nv_,
                           w_.partials);
        double h[2];
        int rc = sums(gv_, 2, h);
        if (rc) return rc;
        *sum_l1 = h[0];
        *sum_ul2 = h[1];
        return SIPO_OK;
    }
    struct Kkt {
        double eps_p, eps_d, eps_gap, p, d, r_p, r_d;
        double rel() const { return std::max(eps_p, std::max(eps_d, eps_gap)); }
        double merit() const { return std::sqrt(eps_p * eps_p + eps_d * eps_d + eps_gap * eps_gap); }
    };
    int kkt(const T *y, const T *D, double u, double v, const T *lu, const T *ll, const T *z, Kkt *out);
    int setup_common();
    int power_norm(int iters, double *nrm);
    int farkas(const T *alu, const T *all, const T *blu, const T *bll, double tol, bool *ok);
    int iteration(bool check);
    int run_block(int nblk);
};

// KKT at (y, D, u, v, lambda); z must hold lambda_up - lambda_lo.  Uses q as scratch.
template <typename T>
int Solver<T>::kkt(const T *y, const T *D, double u, double v, const T *lu, const T *ll, const T *z, Kkt *out) {
    hipLaunchKernelGGL((k_kkt_vox<T>), dim3(gv_), dim3(kThreads), 0, s_, D, lu, ll, lab_, lo_, hi_, c_, u, v, nv_,
                       w_.partials);
    double hv[4];
    int rc = sums(gv_, 4, hv);
    if (rc) return rc;
    rc = adjoint(z, V(w_.q));
    if (rc) return rc;
    hipLaunchKernelGGL((k_kkt_ray<T>), dim3(gs_), dim3(kThreads), 0, s_, (const T *)w_.q, y, act_, ns_, w_.partials);
    double hr[2];
    rc = sums(gs_, 2, hr);
    if (rc) return rc;
    double rp2 = hv[0] + hr[1];
    if (c_.u_free && u < 0) rp2 += u * u;
    if (c_.v_free && v < 0) rp2 += v * v;
    double rd2 = hr[0];
    if (c_.u_free) { const double r = c_.w1 - hv[2]; if (r < 0) rd2 += r * r; }
    if (c_.v_free) { const double r = c_.w2 - hv[3]; if (r < 0) rd2 += r * r; }
    const double pobj = (c_.u_free ? c_.w1 * u : 0.0) + (c_.v_free ? c_.w2 * v : 0.0);
    double dobj = hv[1];
    if (!c_.u_free) dobj -= c_.h * hv[2];
    if (!c_.v_free) dobj -= hv[3];
    out->r_p = std::sqrt(rp2);
    out->r_d = std::sqrt(rd2);
    out->eps_p = out->r_p / (1.0 + h_norm_);
    out->eps_d = out->r_d / (1.0 + c_norm_);
    out->eps_gap = std::fabs(pobj - dobj) / (1.0 + std::fabs(pobj) + std::fabs(dobj));
    out->p = pobj;
    out->d = dobj;
    return SIPO_OK;
}

template <typename T>
int Solver<T>::setup_common() {
    if (t3_) {
        int rc = launch_sino_to_t(p_, pb_.y, y_, s_);
        if (!rc) rc = launch_mask_to_t(p_, pb_.act, (uint8_t *)act_, s_);
        if (rc) return rc;
    }
    hipLaunchKernelGGL((k_project_y<T>), dim3(gs_), dim3(kThreads), 0, s_, y_, act_, ns_);
    double l1, ul2;
    int rc = lambda_z(lu_, ll_, V(w_.z), &l1, &ul2);
    if (rc) return rc;
    // R = K P^T 1_act -> dual scalings; region sizes, ||h||
    hipLaunchKernelGGL((k_colweight<T>), dim3(gv_), dim3(kThreads), 0, s_, V(w_.tmp2), lab_, nv_);
    hipLaunchKernelGGL((k_act_to_float<T>), dim3(gs_), dim3(kThreads), 0, s_, V(w_.q), act_, ns_);
    rc = dose((const T *)w_.q, V(w_.Dt));
    if (rc) return rc;
    hipLaunchKernelGGL((k_row_scaling<T>), dim3(gv_), dim3(kThreads), 0, s_, (const T *)w_.Dt, V(w_.s_up),
                       V(w_.s_lo), lab_, lo_, hi_, c_, nv_, w_.partials);
    double hs[4];
    rc = sums(gv_, 4, hs);
    if (rc) return rc;
    Tu_ = (c_.u_free && hs[0] > 0) ? 1.0 / hs[0] : 0.0;
    Tv_ = (c_.v_free && hs[1] > 0) ? 1.0 / hs[1] : 0.0;
    h_norm_ = std::sqrt(hs[2]);
    c_norm_ = std::hypot(c_.u_free ? c_.w1 : 0.0, c_.v_free ? c_.w2 : 0.0);
    // primal scaling T_j = 1 / (P K w)_j
    rc = adjoint((const T *)w_.tmp2, V(w_.Tj));
    if (rc) return rc;
    hipLaunchKernelGGL((k_inv_colsum<T>), dim3(gs_), dim3(kThreads), 0, s_, V(w_.Tj), act_, ns_);
    // D = K P^T y
    rc = dose(y_, V(w_.D));
    if (rc) return rc;
    std::memset(&hs_, 0, sizeof(hs_));
    hs_.u = c_.u_free ? std::max(0.0, pb_.u0) : c_.h;
    hs_.v = c_.v_free ? std::max(0.0, pb_.v0) : 1.0;
    hs_.sums[0] = l1;
    hs_.sums[1] = ul2;
    return SIPO_OK;
}

template <typename T>
int Solver<T>::power_norm(int iters, double *nrm) {
    T *y = V(w_.y0);   // scratch sinogram
    hipLaunchKernelGGL((k_act_to_float<T>), dim3(gs_), dim3(kThreads), 0, s_, y, act_, ns_);
    hipLaunchKernelGGL((k_pi_mask<T>), dim3(gs_), dim3(kThreads), 0, s_, y, (const T *)y, act_, ns_, w_.partials);
    double yy;
    int rc = sums(gs_, 1, &yy);
    if (rc) return rc;
    double u = c_.u_free ? 1.0 : 0.0, v = c_.v_free ? 1.0 : 0.0;
    double nr = std::sqrt(yy + u * u + v * v);
    if (nr == 0) { *nrm = 0; return SIPO_OK; }
    hipLaunchKernelGGL((k_scale<T>), dim3(gs_), dim3(kThreads), 0, s_, y, 1.0 / nr, ns_);
    u /= nr;
    v /= nr;
    double lam = 0.0;
    for (int it = 0; it < iters; ++it) {
        rc = dose(y, V(w_.Dt));
        if (rc) return rc;
        hipLaunchKernelGGL((k_pi_rows<T>), dim3(gv_), dim3(kThreads), 0, s_, (const T *)w_.Dt, V(w_.tmp2), lab_, hi_,
                           c_, u, v, nv_, w_.partials);
        double rs[2];
        rc = sums(gv_, 2, rs);
        if (rc) return rc;
        rc = adjoint((const T *)w_.tmp2, V(w_.q));
        if (rc) return rc;
        hipLaunchKernelGGL((k_pi_mask<T>), dim3(gs_), dim3(kThreads), 0, s_, y, (const T *)w_.q, act_, ns_,
                           w_.partials);
        rc = sums(gs_, 1, &yy);
        if (rc) return rc;
        const double gu = c_.u_free ? -rs[0] : 0.0, gv = c_.v_free ? -rs[1] : 0.0;
        lam = std::sqrt(yy + gu * gu + gv * gv);
        if (lam == 0) break;
        hipLaunchKernelGGL((k_scale<T>), dim3(gs_), dim3(kThreads), 0, s_, y, 1.0 / lam, ns_);
        u = gu / lam;
        v = gv / lam;
    }
    *nrm = std::sqrt(lam);
    return SIPO_OK;
}

// Farkas test of the candidate d = max(a - b, 0): scaled to dual objective 1, every
// reduced-cost violation must be <= tol.  Uses tmp2 (z_d) and q.
template <typename T>
int Solver<T>::farkas(const T *alu, const T *all, const T *blu, const T *bll, double tol, bool *ok) {
    *ok = false;
    hipLaunchKernelGGL((k_ray_candidate<T>), dim3(gv_), dim3(kThreads), 0, s_, alu, all, blu, bll, V(w_.tmp2), lab_,
                       lo_, hi_, c_, nv_, w_.partials);
    double r[4];
    int rc = sums(gv_, 4, r);
    if (rc) return rc;
    double ray_obj = r[0];
    if (!c_.u_free) ray_obj -= c_.h * r[1];
    if (!c_.v_free) ray_obj -= r[2];
    if (!(ray_obj > 0) || !(r[3] > 0)) return SIPO_OK;
    const double worst_u = c_.u_free ? r[1] / ray_obj : 0.0;
    const double worst_v = c_.v_free ? r[2] / ray_obj : 0.0;
    if (std::max(worst_u, worst_v) > tol) return SIPO_OK;
    rc = adjoint((const T *)w_.tmp2, V(w_.q));
    if (rc) return rc;
    hipLaunchKernelGGL((k_ray_check<T>), dim3(gs_), dim3(kThreads), 0, s_, (const T *)w_.q, act_, ns_, w_.partials);
    hipLaunchKernelGGL(finish_max, dim3(1), dim3(kThreads), 0, s_, w_.partials, gs_, w_.scal->sums);
    double m[2];
    SIPO_HIP(hipMemcpyAsync(m, w_.scal->sums, sizeof(m), hipMemcpyDeviceToHost, s_));
    SIPO_HIP(hipStreamSynchronize(s_));
    *ok = m[0] / ray_obj <= tol;
    return SIPO_OK;
}

// One iteration: t = T(z), z <- Halpern update.  On check iterations t.lambda and the
// pre-step lambda are written out.
template <typename T>
int Solver<T>::iteration(bool check) {
    const bool hal = o_.mode == SIPO_PDHG_RESTARTED;
    prof_on_ = o_.profile != 0;
    int rc = mark(-1);   // start of this iteration's timeline segment
    if (!rc) rc = adjoint((const T *)w_.z, V(w_.q));
    if (rc) return rc;
    hipLaunchKernelGGL((k_primal<T>), dim3(gs_), dim3(kThreads), 0, s_, y_, V(w_.yt), (const T *)w_.q,
                       hal ? (const T *)w_.Tj : (const T *)nullptr, act_, hal ? (const T *)w_.y0 : (const T *)nullptr,
                       (const DevScal *)w_.scal, ns_);
    rc = mark(SIPO_PHASE_PRIMAL);
    if (!rc) rc = dose((const T *)w_.yt, V(w_.Dt));
    if (rc) return rc;
    hipLaunchKernelGGL((k_dual<T>), dim3(gv_), dim3(kThreads), 0, s_, (const T *)w_.Dt, V(w_.D),
                       hal ? (const T *)w_.D0 : (const T *)nullptr, lu_, ll_,
                       hal ? (const T *)w_.lu0 : (const T *)nullptr, hal ? (const T *)w_.ll0 : (const T *)nullptr,
                       V(w_.z), lab_, lo_, hi_, hal ? (const T *)w_.s_up : (const T *)nullptr,
                       hal ? (const T *)w_.s_lo : (const T *)nullptr, check ? V(w_.lut) : (T *)nullptr,
                       check ? V(w_.llt) : (T *)nullptr, check ? V(w_.luo) : (T *)nullptr,
                       check ? V(w_.llo) : (T *)nullptr, (const DevScal *)w_.scal, c_, nv_, w_.partials);
    rc = mark(SIPO_PHASE_DUAL);
    if (rc) return rc;
    hipLaunchKernelGGL(k_scalars, dim3(1), dim3(kThreads), 0, s_, w_.partials, gv_, w_.scal, c_);
    rc = mark(SIPO_PHASE_SCALARS);
    prof_on_ = false;
    return rc;
}

// nblk iterations, the last one a check iteration; captured once into a graph when requested.
template <typename T>
int Solver<T>::run_block(int nblk) {
    if (!o_.use_graph) {
        for (int j = 0; j < nblk; ++j) {
            int rc = iteration(j == nblk - 1);
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
    SIPO_HIP(hipGraphLaunch(graph_exec_, s_));
    return SIPO_OK;
}

template <typename T>
int Solver<T>::run(sipo_pdhg_result *res) {
    auto t0 = std::chrono::steady_clock::now();
    std::memset(res, 0, sizeof(*res));
    int rc = setup_common();
    if (rc) return rc;
    const bool hal = o_.mode == SIPO_PDHG_RESTARTED;
    double omega = 1.0;
    const double eta = o_.eta > 0 ? o_.eta : 0.95;
    double tau = o_.tau, sigma = o_.sigma;
    if (!hal) {
        if (!(tau > 0 && sigma > 0)) {
            double nrm = 0;
            rc = power_norm(o_.power_iters > 0 ? o_.power_iters : 100, &nrm);
            if (rc) return rc;
            if (!(nrm > 0)) return fail(SIPO_E_INVALID, "operator norm is zero (no active rays or no regions)");
            tau = sigma = 0.9 / nrm;
        }
        hs_.tau_fac = tau;
        hs_.sig_fac = sigma;
        hs_.tau_u = tau;
        hs_.tau_v = tau;
        hs_.halpern = 0.0;
        hs_.rho = 0.0;
    } else {
        hs_.tau_fac = eta / omega;
        hs_.sig_fac = eta * omega;
        hs_.tau_u = eta * Tu_ / omega;
        hs_.tau_v = eta * Tv_ / omega;
        hs_.halpern = 1.0;
        hs_.rho = 1.0;
    }
    hs_.u0 = hs_.u;
    hs_.v0 = hs_.v;
    double last_u = hs_.u, last_v = hs_.v;
    rc = put_scal();
    if (rc) return rc;
    hipLaunchKernelGGL(k_scalars_init, dim3(1), dim3(1), 0, s_, w_.scal, c_);
    if (hal) {
        // anchor, restart point and snapshot start at the initial point
        copy(V(w_.y0), (const T *)y_, ns_, gs_);
        copy(V(w_.ylast), (const T *)y_, ns_, gs_);
        copy(V(w_.D0), (const T *)w_.D, nv_, gv_);
        for (void *dst : {w_.lu0, w_.lul, w_.snap_u}) copy(V(dst), (const T *)lu_, nv_, gv_);
        for (void *dst : {w_.ll0, w_.lll, w_.snap_l}) copy(V(dst), (const T *)ll_, nv_, gv_);
    }
    SIPO_LAUNCHED("pdhg setup");

    const int check = hal ? std::max(1, o_.check_every) : o_.max_iters;
    const double itol = o_.infeas_tol > 0 ? o_.infeas_tol : 1e-6;
    int status = SIPO_ITER_LIMIT, restarts = 0, it = 0, k_restart = 0;
    Kkt kc{};
    double m_anchor = 0, m_prev = 1e300;
    bool have_t = false;          // lut/llt/yt/Dt/ut_done hold a PDHG output t
    const T *cert_a_u = nullptr, *cert_a_l = nullptr, *cert_b_u = nullptr, *cert_b_l = nullptr;
    if (hal) {
        Kkt k0{};
        rc = kkt(y_, (const T *)w_.D, hs_.u, hs_.v, lu_, ll_, (const T *)w_.z, &k0);
        if (rc) return rc;
        m_anchor = k0.merit();
    }
    while (it < o_.max_iters) {
        const int nblk = std::min(check, o_.max_iters - it);
        rc = run_block(nblk);
        if (!rc) rc = flush_profile();
        if (rc) return rc;
        it += nblk;
        have_t = true;
        if (!hal) break;
        rc = get_scal();
        if (rc) return rc;
        if (!std::isfinite(hs_.u) || !std::isfinite(hs_.v) || !std::isfinite(hs_.sum_l1) ||
            !std::isfinite(hs_.sum_Ul2)) {
            status = SIPO_NUMERICAL;
            break;
        }
        // KKT of the PDHG output t; z_lambda(t) into tmp2
        double tl1, tul2;
        rc = lambda_z(V(w_.lut), V(w_.llt), V(w_.tmp2), &tl1, &tul2);
        if (rc) return rc;
        rc = kkt((const T *)w_.yt, (const T *)w_.Dt, hs_.ut_done, hs_.vt_done, (const T *)w_.lut,
                 (const T *)w_.llt, (const T *)w_.tmp2, &kc);
        if (rc) return rc;
        if (!std::isfinite(kc.r_p) || !std::isfinite(kc.r_d)) { status = SIPO_NUMERICAL; break; }
        if (kc.rel() <= o_.tol) { status = SIPO_OPTIMAL; break; }
        bool inf = false;
        rc = farkas((const T *)w_.lut, (const T *)w_.llt, (const T *)w_.luo, (const T *)w_.llo, itol, &inf);
        if (rc) return rc;
        if (inf) {
            cert_a_u = (const T *)w_.lut; cert_a_l = (const T *)w_.llt;
            cert_b_u = (const T *)w_.luo; cert_b_l = (const T *)w_.llo;
        } else {
            rc = farkas((const T *)w_.lut, (const T *)w_.llt, (const T *)w_.snap_u, (const T *)w_.snap_l, itol, &inf);
            if (rc) return rc;
            if (inf) {
                cert_a_u = (const T *)w_.lut; cert_a_l = (const T *)w_.llt;
                cert_b_u = (const T *)w_.snap_u; cert_b_l = (const T *)w_.snap_l;
            }
        }
        if (inf) { status = SIPO_PRIMAL_INFEASIBLE; break; }
        copy(V(w_.snap_u), (const T *)w_.lut, nv_, gv_);
        copy(V(w_.snap_l), (const T *)w_.llt, nv_, gv_);
        const double m = kc.merit();
        if (!(m <= 0.2 * m_anchor || (m <= 0.8 * m_anchor && m > m_prev) ||
              (double)(it - k_restart) >= 0.36 * (double)it)) {
            m_prev = m;
            continue;
        }
        // ---- restart at t: movement since the previous restart -> primal weight
        double dy2, dlu2, dll2;
        hipLaunchKernelGGL((k_wdist<T>), dim3(gs_), dim3(kThreads), 0, s_, (const T *)w_.yt, (const T *)w_.ylast,
                           (const T *)w_.Tj, ns_, w_.partials);
        rc = sums(gs_, 1, &dy2);
        if (rc) return rc;
        hipLaunchKernelGGL((k_wdist<T>), dim3(gv_), dim3(kThreads), 0, s_, (const T *)w_.lut, (const T *)w_.lul,
                           (const T *)w_.s_up, nv_, w_.partials);
        rc = sums(gv_, 1, &dlu2);
        if (rc) return rc;
        hipLaunchKernelGGL((k_wdist<T>), dim3(gv_), dim3(kThreads), 0, s_, (const T *)w_.llt, (const T *)w_.lll,
                           (const T *)w_.s_lo, nv_, w_.partials);
        rc = sums(gv_, 1, &dll2);
        if (rc) return rc;
        const double du = hs_.ut_done - last_u, dv = hs_.vt_done - last_v;
        const double dx = std::sqrt(dy2 + (Tu_ > 0 ? du * du / Tu_ : 0.0) + (Tv_ > 0 ? dv * dv / Tv_ : 0.0));
        const double dl = std::sqrt(dlu2 + dll2);
        if (dx > 1e-10 && dl > 1e-10) omega = std::exp(0.5 * std::log(dl / dx) + 0.5 * std::log(omega));
        // z, z0 and the restart point become t
        for (void *dst : {(void *)y_, w_.y0, w_.ylast}) copy(V(dst), (const T *)w_.yt, ns_, gs_);
        for (void *dst : {(void *)lu_, w_.lu0, w_.lul}) copy(V(dst), (const T *)w_.lut, nv_, gv_);
        for (void *dst : {(void *)ll_, w_.ll0, w_.lll}) copy(V(dst), (const T *)w_.llt, nv_, gv_);
        for (void *dst : {w_.D, w_.D0}) copy(V(dst), (const T *)w_.Dt, nv_, gv_);
        double l1, ul2;
        rc = lambda_z(lu_, ll_, V(w_.z), &l1, &ul2);
        if (rc) return rc;
        hs_.u = hs_.u0 = last_u = hs_.ut_done;
        hs_.v = hs_.v0 = last_v = hs_.vt_done;
        hs_.sums[0] = l1;
        hs_.sums[1] = ul2;
        hs_.tau_fac = eta / omega;
        hs_.sig_fac = eta * omega;
        hs_.tau_u = eta * Tu_ / omega;
        hs_.tau_v = eta * Tv_ / omega;
        rc = put_scal();
        if (rc) return rc;
        hipLaunchKernelGGL(k_scalars_init, dim3(1), dim3(1), 0, s_, w_.scal, c_);
        m_anchor = m;
        m_prev = 1e300;
        k_restart = it;
        ++restarts;
    }
    // ---------------- returned point: the PDHG output t (restarted) or z = t (plain)
    rc = get_scal();
    if (rc) return rc;
    double u = hs_.u, v = hs_.v;
    if (hal && have_t) {
        u = hs_.ut_done;
        v = hs_.vt_done;
        copy(y_, (const T *)w_.yt, ns_, gs_);
        copy(V(w_.D), (const T *)w_.Dt, nv_, gv_);
        if (status == SIPO_PRIMAL_INFEASIBLE) {
            hipLaunchKernelGGL((k_certificate<T>), dim3(gv_), dim3(kThreads), 0, s_, lu_, ll_, cert_a_u, cert_a_l,
                               cert_b_u, cert_b_l, lab_, nv_);
        } else {
            copy(lu_, (const T *)w_.lut, nv_, gv_);
            copy(ll_, (const T *)w_.llt, nv_, gv_);
        }
    }
    if (status == SIPO_ITER_LIMIT || status == SIPO_NUMERICAL || !hal) {
        hipLaunchKernelGGL((k_lambda_z<T>), dim3(gv_), dim3(kThreads), 0, s_, lu_, ll_, V(w_.z), lab_, hi_, c_, nv_,
                           w_.partials);
        rc = kkt(y_, (const T *)w_.D, u, v, lu_, ll_, (const T *)w_.z, &kc);
        if (rc) return rc;
    }
    if (pb_.dose_out) copy((T *)pb_.dose_out, (const T *)w_.D, nv_, gv_);
    if (t3_) {
        rc = launch_sino_from_t(p_, y_, pb_.y, 0, s_);
        if (rc) return rc;
    }
    SIPO_LAUNCHED("pdhg finish");
    SIPO_HIP(hipStreamSynchronize(s_));
    res->status = status;
    res->iters = it;
    res->restarts = restarts;
    res->primal_obj = kc.p;
    res->dual_obj = kc.d;
    res->rel_primal = kc.eps_p;
    res->rel_dual = kc.eps_d;
    res->rel_gap = kc.eps_gap;
    res->u = u;
    res->v = v;
    res->tau = tau;
    res->sigma = sigma;
    res->omega = omega;
    res->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (int ph = 0; ph < SIPO_NUM_PHASES; ++ph) {
        res->phase_ms[ph] = phase_ms_[ph];
        res->phase_launches[ph] = phase_n_[ph];
    }
    return SIPO_OK;
}

static int validate(const sipo_problem &pb, const sipo_pdhg_options &o, int idx) {
    int rc = check_plan(pb.plan);
    if (rc) return rc;
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
    return SIPO_OK;
}

}  // namespace sipo

using namespace sipo;

extern "C" {

size_t sipo_pdhg_workspace_size(const sipo_problem *probs, int32_t n, const sipo_pdhg_options *) {
    if (!probs || n < 1) return 0;
    size_t m = 0;
    for (int i = 0; i < n; ++i)
        if (probs[i].plan) m = std::max(m, layout(probs[i], nullptr, nullptr));
    return m;
}

int sipo_pdhg_solve(const sipo_problem *probs, int32_t n, const sipo_pdhg_options *opts, void *workspace,
                    size_t ws_bytes, sipo_pdhg_result *results, void *stream) {
    SIPO_REQUIRE(probs && opts && results && n >= 1, "NULL argument or n < 1");
    for (int i = 0; i < n; ++i) {
        int rc = validate(probs[i], *opts, i);
        if (rc) return rc;
    }
    const size_t need = sipo_pdhg_workspace_size(probs, n, opts);
    SIPO_REQUIRE(workspace != nullptr, "workspace is NULL");
    if (ws_bytes < need) return fail(SIPO_E_WORKSPACE, "workspace of %zu bytes < %zu required", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    SIPO_REQUIRE(!(opts->use_graph && s == nullptr), "graph capture needs a non-default stream");
    for (int i = 0; i < n; ++i) {
        Workspace w;
        layout(probs[i], &w, (char *)workspace);
        int rc = probs[i].plan->dtype == SIPO_F64 ? Solver<double>(probs[i], *opts, w, s).run(&results[i])
                                                  : Solver<float>(probs[i], *opts, w, s).run(&results[i]);
        if (rc) return rc;
    }
    return SIPO_OK;
}

}  // extern "C"
