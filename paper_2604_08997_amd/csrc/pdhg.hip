// Matrix-free PDHG for the unified Charnes-Cooper LP (Sec. 2.8, Supp. 6.1).
//
// Saddle problem  min_{x in X} max_{lambda >= 0} c^T x + lambda^T (G x - h)
// with x = (y, u, v), D = K P^T y and the rows (band: D - u_bar, gel: D - v_bar U,
// gel: L - D).  One iteration (Chambolle-Pock, primal first):
//
//   q   = P K z,  z = lambda_up[band | gel] - lambda_lo[gel]          (Eq. 51)
//   y+  = act ? max(0, y - tau_j q) : 0                               (Eq. 50)
//   u+  = max(0, u - tau_u (w1 - sum lambda1)),  v+ likewise          (Eq. 48-49)
//   D+  = K P^T y+,  Dbar = 2 D+ - D,  ubar = 2 u+ - u,  vbar = 2 v+ - v
//   lambda_up <- max(0, lambda_up + s_i (Dbar - ubar | vbar U))       band | gel
//   lambda_lo <- max(0, lambda_lo + s_i (L - Dbar))                   gel
//
// Plain mode: scalar tau = sigma = 0.9 / ||G|| (FP64 power iteration).
// Restarted mode: diagonal steps T_j = 1 / colsum_j(|G|), S_i = 1 / rowsum_i(|G|)
// with a primal weight omega (tau = eta T / omega, sigma = eta omega S), uniform
// averages since the last restart, KKT checks every check_every iterations on
// the current and the averaged iterate, restarts to the better of the two
// (sufficient 0.2 / necessary 0.8 / artificial 0.36), omega updated from the
// movement between restarts, and the dual iterate difference over each check
// window tested as a Farkas certificate.
//
// Everything that changes from one iteration to the next lives in a device
// scalar block, so an iteration is a fixed sequence of launches with fixed
// arguments (graph-capturable).  Reductions are two-level (per-block FP64
// partials, then one block summing them in a fixed order): deterministic.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

#include "sipo_internal.hpp"

namespace sipo {

constexpr int kRedBlocks = 1024;   // upper bound on reduction blocks
constexpr int kNS = 8;             // sums carried per reduction
constexpr int kThreads = 256;

// Device scalar block (FP64): all iteration-varying values.
struct DevScal {
    double u, v;              // current u^k, v^k
    double u_next, v_next;    // u^{k+1}, v^{k+1}
    double ubar, vbar;        // extrapolated scalars for the dual update
    double tau_fac, sig_fac;  // array step factors (eta/omega, eta*omega) or plain tau, sigma
    double tau_u, tau_v;      // scalar primal steps
    double avg_w, n_avg;      // weight of the current iterate in the running average
    double u_avg, v_avg;
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

// Sum per-block partials (fixed order) into dst[0..NS).
__global__ void finish_sums(const double *__restrict__ partials, int nblocks, double *dst, int ns) {
    const int k = threadIdx.x;
    if (k < ns) {
        double s = 0.0;
        for (int b = 0; b < nblocks; ++b) s += partials[b * kNS + k];
        dst[k] = s;
    }
}

static int red_blocks(size_t n) { return (int)std::min<size_t>((n + kThreads * 4 - 1) / (kThreads * 4), kRedBlocks); }

#define GRID_LOOP(i, n) for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < (n); i += (size_t)gridDim.x * blockDim.x)

template <typename T>
__device__ __forceinline__ T ld_or(const T *p, size_t i, double s) { return p ? p[i] : (T)s; }

// ------------------------------------------------------------- setup kernels
// y <- act ? max(y, 0) : 0  (warm start sanitised onto X)
template <typename T>
__global__ void k_project_y(T *y, const uint8_t *act, size_t n) {
    GRID_LOOP(i, n) y[i] = act[i] ? (y[i] > (T)0 ? y[i] : (T)0) : (T)0;
}

// lambda sanitised onto its regions and made >= 0; z = lambda_up - lambda_lo; sums of lambda.
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

// S_up = 1/(R + [band, u free] + [gel, v free] U), S_lo = [gel] 1/R; sums |band|, sum_gel U, ||h||^2 pieces
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
// y+ = act ? max(0, y - tau q) : 0, with tau = tau_fac * T_j (or tau_fac); running average of y.
template <typename T>
__global__ void k_primal(T *__restrict__ y, const T *__restrict__ q, const T *__restrict__ Tj,
                         const uint8_t *__restrict__ act, T *__restrict__ y_avg, const DevScal *__restrict__ sc,
                         size_t n) {
    const T tf = (T)sc->tau_fac;
    const T aw = (T)sc->avg_w;
    GRID_LOOP(i, n) {
        T yn = (T)0;
        if (act[i]) {
            const T t = Tj ? tf * Tj[i] : tf;
            yn = y[i] - t * q[i];
            yn = yn > (T)0 ? yn : (T)0;
        }
        y[i] = yn;
        if (y_avg) y_avg[i] += aw * (yn - y_avg[i]);
    }
}

// Dual update on voxels; writes lambda, z, averages; block sums of lambda1 and U lambda2.
template <typename T>
__global__ void k_dual(const T *__restrict__ Dn, const T *__restrict__ Do, T *__restrict__ lu, T *__restrict__ ll,
                       T *__restrict__ z, const uint8_t *__restrict__ lab, const T *__restrict__ lo,
                       const T *__restrict__ hi, const T *__restrict__ s_up, const T *__restrict__ s_lo,
                       T *__restrict__ lu_avg, T *__restrict__ ll_avg, const DevScal *__restrict__ sc, LPConst c,
                       size_t n, double *partials) {
    const double sf = sc->sig_fac;
    const T ub = (T)(c.u_free ? sc->ubar : c.h);
    const T vb = (T)(c.v_free ? sc->vbar : 1.0);
    const T aw = (T)sc->avg_w;
    double acc[kNS] = {0, 0, 0, 0, 0, 0, 0, 0};
    GRID_LOOP(i, n) {
        const uint8_t L = lab[i];
        if (L == 0) continue;
        const T Db = (T)2 * Dn[i] - Do[i];
        const T su = s_up ? (T)sf * s_up[i] : (T)sf;
        T a = lu[i] + su * (Db - (L == 1 ? ub : vb * ld_or(hi, i, c.hi_s)));
        a = a > (T)0 ? a : (T)0;
        lu[i] = a;
        T zz = a;
        if (lu_avg) lu_avg[i] += aw * (a - lu_avg[i]);
        if (L == 1) {
            acc[0] += (double)a;
        } else {
            const T sl = s_lo ? (T)sf * s_lo[i] : (T)sf;
            T b = ll[i] + sl * (ld_or(lo, i, c.lo_s) - Db);
            b = b > (T)0 ? b : (T)0;
            ll[i] = b;
            zz = a - b;
            if (ll_avg) ll_avg[i] += aw * (b - ll_avg[i]);
            acc[1] += (double)ld_or(hi, i, c.hi_s) * (double)a;
        }
        z[i] = zz;
    }
    block_sums<kNS>(acc, partials);
}

// One block: finish the lambda sums and roll the scalars for the next iteration.
__global__ void k_scalars(const double *__restrict__ partials, int nblocks, DevScal *sc, LPConst c) {
    __shared__ double s[2];
    if (threadIdx.x < 2) {
        double a = 0.0;
        for (int b = 0; b < nblocks; ++b) a += partials[b * kNS + threadIdx.x];
        s[threadIdx.x] = a;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double w = sc->avg_w;
    // the iterate just completed is (u_next, v_next) = (u^{k+1}, v^{k+1})
    sc->u = sc->u_next;
    sc->v = sc->v_next;
    sc->u_avg += w * (sc->u - sc->u_avg);
    sc->v_avg += w * (sc->v - sc->v_avg);
    sc->n_avg += 1.0;
    sc->avg_w = 1.0 / sc->n_avg;
    sc->sum_l1 = s[0];
    sc->sum_Ul2 = s[1];
    if (c.u_free) sc->u_next = fmax(0.0, sc->u - sc->tau_u * (c.w1 - s[0]));
    else sc->u_next = c.h;
    if (c.v_free) sc->v_next = fmax(0.0, sc->v - sc->tau_v * (c.w2 - s[1]));
    else sc->v_next = 1.0;
    sc->ubar = 2.0 * sc->u_next - sc->u;
    sc->vbar = 2.0 * sc->v_next - sc->v;
}

// Initial roll: given sums of lambda^0 in sc->sums[0..1], set u_next, ubar for iteration 0.
__global__ void k_scalars_init(DevScal *sc, LPConst c) {
    sc->sum_l1 = sc->sums[0];
    sc->sum_Ul2 = sc->sums[1];
    sc->u_next = c.u_free ? fmax(0.0, sc->u - sc->tau_u * (c.w1 - sc->sum_l1)) : c.h;
    sc->v_next = c.v_free ? fmax(0.0, sc->v - sc->tau_v * (c.w2 - sc->sum_Ul2)) : 1.0;
    sc->ubar = 2.0 * sc->u_next - sc->u;
    sc->vbar = 2.0 * sc->v_next - sc->v;
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

// Farkas candidate: d = max(lam - snap, 0) on regions -> z_d; sums for the ray objective.
// [0] sum L d3, [1] sum_band d1, [2] sum_gel U d2, [3] sum |d| (l1)
template <typename T>
__global__ void k_ray_candidate(const T *lu, const T *ll, const T *su, const T *sl, T *zd, const uint8_t *lab,
                                const T *lo, const T *hi, LPConst c, size_t n, double *partials) {
    double acc[kNS] = {0, 0, 0, 0, 0, 0, 0, 0};
    GRID_LOOP(i, n) {
        const uint8_t L = lab[i];
        T zz = 0;
        if (L) {
            T a = lu[i] - su[i];
            a = a > (T)0 ? a : (T)0;
            zz = a;
            acc[3] += (double)a;
            if (L == 1) acc[1] += (double)a;
            else {
                T b = ll[i] - sl[i];
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

// Certificate output: lambda_up <- max(lambda_up - snap_up, 0), lambda_lo <- max(lambda_lo - snap_lo, 0) on regions.
template <typename T>
__global__ void k_certificate(T *lu, T *ll, const T *su, const T *sl, const uint8_t *lab, size_t n) {
    GRID_LOOP(i, n) {
        const uint8_t L = lab[i];
        T a = L ? lu[i] - su[i] : (T)0;
        T b = (L == 2) ? ll[i] - sl[i] : (T)0;
        lu[i] = a > (T)0 ? a : (T)0;
        ll[i] = b > (T)0 ? b : (T)0;
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

__global__ void finish_max(const double *__restrict__ partials, int nblocks, double *dst) {
    if (threadIdx.x < 2) {
        double m = 0.0;
        for (int b = 0; b < nblocks; ++b) m = fmax(m, partials[b * kNS + threadIdx.x]);
        dst[threadIdx.x] = m;
    }
}

// power iteration: rows of G x for x = (y, u, v) with D = K P^T y -> z = G^T-row combination,
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

// weighted movement norms: [0] sum (a-b)^2 / w over w > 0
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
    // sinogram-sized
    void *q, *Tj, *y_avg, *y_anchor;
    // volume-sized
    void *D, *Dn, *z, *tmp, *tmp2, *s_up, *s_lo, *lu_avg, *ll_avg, *lu_anchor, *ll_anchor, *lu_snap, *ll_snap;
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
    Workspace w;
    w.q = take(sb); w.Tj = take(sb); w.y_avg = take(sb); w.y_anchor = take(sb);
    w.D = take(vb); w.Dn = take(vb); w.z = take(vb); w.tmp = take(vb); w.tmp2 = take(vb);
    w.s_up = take(vb); w.s_lo = take(vb); w.lu_avg = take(vb); w.ll_avg = take(vb);
    w.lu_anchor = take(vb); w.ll_anchor = take(vb); w.lu_snap = take(vb); w.ll_snap = take(vb);
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
        act_ = pb.act;
        lo_ = (const T *)pb.lo;
        hi_ = (const T *)pb.hi;
        y_ = (T *)pb.y;
        lu_ = (T *)pb.lam_up;
        ll_ = (T *)pb.lam_lo;
        gv_ = std::min<size_t>((nv_ + kThreads * 4 - 1) / (kThreads * 4), kRedBlocks);
        gs_ = std::min<size_t>((ns_ + kThreads * 4 - 1) / (kThreads * 4), kRedBlocks);
        gv_ = std::max(gv_, 1);
        gs_ = std::max(gs_, 1);
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
    const T *lo_, *hi_;
    T *y_, *lu_, *ll_;
    double h_norm_ = 0, c_norm_ = 0;
    double Tu_ = 0, Tv_ = 0;
    double anchor_u_ = 0, anchor_v_ = 0;
    DevScal hs_{};

    // operators
    int dose(const T *y, T *out) {   // out = K P^T y  (uses tmp when K != I)
        if (!p_->has_psf) return launch_backproject(p_, y, out, 0, s_);
        int rc = launch_backproject(p_, y, w_.tmp, 0, s_);
        return rc ? rc : launch_blur(p_, w_.tmp, out, s_);
    }
    int adjoint(const T *z, T *out) {   // out = P K z
        if (!p_->has_psf) return launch_project(p_, z, out, 0, s_);
        int rc = launch_blur(p_, z, w_.tmp, s_);
        return rc ? rc : launch_project(p_, w_.tmp, out, 0, s_);
    }
    int sums(int nblocks, int ns, double *host) {
        hipLaunchKernelGGL(finish_sums, dim3(1), dim3(64), 0, s_, w_.partials, nblocks, w_.scal->sums, ns);
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
    // KKT at (y, D, u, v, lambda); z must hold lambda_up - lambda_lo.  Uses q as scratch.
    int kkt(const T *y, const T *D, double u, double v, const T *lu, const T *ll, const T *z, Kkt *out) {
        hipLaunchKernelGGL((k_kkt_vox<T>), dim3(gv_), dim3(kThreads), 0, s_, D, lu, ll, lab_, lo_, hi_, c_, u, v,
                           nv_, w_.partials);
        double hv[4];
        int rc = sums(gv_, 4, hv);
        if (rc) return rc;
        rc = adjoint(z, (T *)w_.q);
        if (rc) return rc;
        hipLaunchKernelGGL((k_kkt_ray<T>), dim3(gs_), dim3(kThreads), 0, s_, (const T *)w_.q, y, act_, ns_,
                           w_.partials);
        double hr[2];
        rc = sums(gs_, 2, hr);
        if (rc) return rc;
        double rp2 = hv[0] + hr[1];
        if (c_.u_free) { const double r = -u; if (r > 0) rp2 += r * r; }
        if (c_.v_free) { const double r = -v; if (r > 0) rp2 += r * r; }
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
    int setup_common();
    int power_norm(int iters, double *nrm);
    int farkas(double tol, T *zd, bool *ok);
};

template <typename T>
int Solver<T>::setup_common() {
    // sanitise the warm start onto X and the regions; z, lambda sums
    hipLaunchKernelGGL((k_project_y<T>), dim3(gs_), dim3(kThreads), 0, s_, y_, act_, ns_);
    double l1, ul2;
    int rc = lambda_z(lu_, ll_, (T *)w_.z, &l1, &ul2);
    if (rc) return rc;
    // region sizes and ||h||
    hipLaunchKernelGGL((k_colweight<T>), dim3(gv_), dim3(kThreads), 0, s_, (T *)w_.tmp2, lab_, nv_);
    // R = K P^T 1_act -> s_up/s_lo (restarted) ; also |band|, sum U, ||h||^2
    hipLaunchKernelGGL((k_act_to_float<T>), dim3(gs_), dim3(kThreads), 0, s_, (T *)w_.q, act_, ns_);
    rc = dose((const T *)w_.q, (T *)w_.Dn);
    if (rc) return rc;
    hipLaunchKernelGGL((k_row_scaling<T>), dim3(gv_), dim3(kThreads), 0, s_, (const T *)w_.Dn, (T *)w_.s_up,
                       (T *)w_.s_lo, lab_, lo_, hi_, c_, nv_, w_.partials);
    double hs[4];
    rc = sums(gv_, 4, hs);
    if (rc) return rc;
    Tu_ = (c_.u_free && hs[0] > 0) ? 1.0 / hs[0] : 0.0;
    Tv_ = (c_.v_free && hs[1] > 0) ? 1.0 / hs[1] : 0.0;
    h_norm_ = std::sqrt(hs[2]);
    c_norm_ = std::hypot(c_.u_free ? c_.w1 : 0.0, c_.v_free ? c_.w2 : 0.0);
    // column scaling T_j = 1 / (P K w)_j
    rc = adjoint((const T *)w_.tmp2, (T *)w_.Tj);
    if (rc) return rc;
    hipLaunchKernelGGL((k_inv_colsum<T>), dim3(gs_), dim3(kThreads), 0, s_, (T *)w_.Tj, act_, ns_);
    // D = K P^T y (current dose)
    rc = dose(y_, (T *)w_.D);
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
    // x = (act, 1, 1) normalised
    T *y = (T *)w_.y_avg;   // scratch sinogram
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
        rc = dose(y, (T *)w_.Dn);
        if (rc) return rc;
        hipLaunchKernelGGL((k_pi_rows<T>), dim3(gv_), dim3(kThreads), 0, s_, (const T *)w_.Dn, (T *)w_.tmp2, lab_,
                           hi_, c_, u, v, nv_, w_.partials);
        double rs[2];
        rc = sums(gv_, 2, rs);
        if (rc) return rc;
        rc = adjoint((const T *)w_.tmp2, (T *)w_.q);
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

// Farkas test of d = max(lambda - snapshot, 0) (see k_ray_candidate); ok = certificate accepted.
template <typename T>
int Solver<T>::farkas(double tol, T *zd, bool *ok) {
    *ok = false;
    hipLaunchKernelGGL((k_ray_candidate<T>), dim3(gv_), dim3(kThreads), 0, s_, (const T *)lu_, (const T *)ll_,
                       (const T *)w_.lu_snap, (const T *)w_.ll_snap, zd, lab_, lo_, hi_, c_, nv_, w_.partials);
    double r[4];
    int rc = sums(gv_, 4, r);
    if (rc) return rc;
    double ray_obj = r[0];
    if (!c_.u_free) ray_obj -= c_.h * r[1];
    if (!c_.v_free) ray_obj -= r[2];
    if (!(ray_obj > 0) || !(r[3] > 0)) return SIPO_OK;
    // scale to ray_obj = 1 and test the reduced costs
    const double worst_u = c_.u_free ? r[1] / ray_obj : 0.0;
    const double worst_v = c_.v_free ? r[2] / ray_obj : 0.0;
    rc = adjoint((const T *)zd, (T *)w_.q);
    if (rc) return rc;
    hipLaunchKernelGGL((k_ray_check<T>), dim3(gs_), dim3(kThreads), 0, s_, (const T *)w_.q, act_, ns_, w_.partials);
    hipLaunchKernelGGL(finish_max, dim3(1), dim3(64), 0, s_, w_.partials, gs_, w_.scal->sums);
    double m[2];
    SIPO_HIP(hipMemcpyAsync(m, w_.scal->sums, sizeof(m), hipMemcpyDeviceToHost, s_));
    SIPO_HIP(hipStreamSynchronize(s_));
    const double worst_q = m[0] / ray_obj;
    const double worst = std::max(worst_q, std::max(worst_u, worst_v));
    *ok = worst <= tol;
    return SIPO_OK;
}

template <typename T>
int Solver<T>::run(sipo_pdhg_result *res) {
    auto t0 = std::chrono::steady_clock::now();
    std::memset(res, 0, sizeof(*res));
    int rc = setup_common();
    if (rc) return rc;
    const bool restarted = o_.mode == SIPO_PDHG_RESTARTED;
    double omega = 1.0;
    const double eta = o_.eta > 0 ? o_.eta : 0.95;
    double tau = o_.tau, sigma = o_.sigma;
    if (!restarted) {
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
    } else {
        hs_.tau_fac = eta / omega;
        hs_.sig_fac = eta * omega;
        hs_.tau_u = eta * Tu_ / omega;
        hs_.tau_v = eta * Tv_ / omega;
    }
    hs_.n_avg = 1.0;
    hs_.avg_w = 1.0;
    hs_.u_avg = hs_.u;
    hs_.v_avg = hs_.v;
    anchor_u_ = hs_.u;
    anchor_v_ = hs_.v;
    rc = put_scal();
    if (rc) return rc;
    hipLaunchKernelGGL(k_scalars_init, dim3(1), dim3(1), 0, s_, w_.scal, c_);
    // averages / anchor / snapshot start at the initial point
    if (restarted) {
        hipLaunchKernelGGL((k_copy<T>), dim3(gs_), dim3(kThreads), 0, s_, (T *)w_.y_avg, (const T *)y_, ns_);
        hipLaunchKernelGGL((k_copy<T>), dim3(gs_), dim3(kThreads), 0, s_, (T *)w_.y_anchor, (const T *)y_, ns_);
        for (auto pr : {std::make_pair(w_.lu_avg, (void *)lu_), std::make_pair(w_.ll_avg, (void *)ll_),
                        std::make_pair(w_.lu_anchor, (void *)lu_), std::make_pair(w_.ll_anchor, (void *)ll_),
                        std::make_pair(w_.lu_snap, (void *)lu_), std::make_pair(w_.ll_snap, (void *)ll_)})
            hipLaunchKernelGGL((k_copy<T>), dim3(gv_), dim3(kThreads), 0, s_, (T *)pr.first, (const T *)pr.second, nv_);
    }
    SIPO_LAUNCHED("pdhg setup");

    T *D = (T *)w_.D, *Dn = (T *)w_.Dn;
    const T *Tj = restarted ? (const T *)w_.Tj : nullptr;
    const T *su = restarted ? (const T *)w_.s_up : nullptr;
    const T *sl = restarted ? (const T *)w_.s_lo : nullptr;
    T *y_avg = restarted ? (T *)w_.y_avg : nullptr;
    T *lu_avg = restarted ? (T *)w_.lu_avg : nullptr;
    T *ll_avg = restarted ? (T *)w_.ll_avg : nullptr;
    const int check = restarted ? std::max(1, o_.check_every) : o_.max_iters;
    Kkt k0{};
    double m_anchor = 0, m_prev = 1e300;
    int k_restart = 0, restarts = 0;
    int status = SIPO_ITER_LIMIT;
    int it = 0;
    bool use_avg_final = false;
    Kkt final_kkt{};
    if (restarted) {
        rc = kkt(y_, D, hs_.u, hs_.v, lu_, ll_, (const T *)w_.z, &k0);
        if (rc) return rc;
        m_anchor = k0.merit();
    }
    while (it < o_.max_iters) {
        const int nblk = std::min(check, o_.max_iters - it);
        for (int j = 0; j < nblk; ++j) {
            rc = adjoint((const T *)w_.z, (T *)w_.q);
            if (rc) return rc;
            hipLaunchKernelGGL((k_primal<T>), dim3(gs_), dim3(kThreads), 0, s_, y_, (const T *)w_.q, Tj, act_, y_avg,
                               (const DevScal *)w_.scal, ns_);
            rc = dose(y_, Dn);
            if (rc) return rc;
            hipLaunchKernelGGL((k_dual<T>), dim3(gv_), dim3(kThreads), 0, s_, (const T *)Dn, (const T *)D, lu_, ll_,
                               (T *)w_.z, lab_, lo_, hi_, su, sl, lu_avg, ll_avg, (const DevScal *)w_.scal, c_, nv_,
                               w_.partials);
            hipLaunchKernelGGL(k_scalars, dim3(1), dim3(64), 0, s_, w_.partials, gv_, w_.scal, c_);
            std::swap(D, Dn);
        }
        SIPO_LAUNCHED("pdhg iteration");
        it += nblk;
        if (!restarted) break;
        // ---------------- check: KKT of current and average
        rc = get_scal();
        if (rc) return rc;
        if (!std::isfinite(hs_.u) || !std::isfinite(hs_.v) || !std::isfinite(hs_.sum_l1) ||
            !std::isfinite(hs_.sum_Ul2)) {
            status = SIPO_NUMERICAL;
            break;
        }
        Kkt kc{}, ka{};
        rc = kkt(y_, D, hs_.u, hs_.v, lu_, ll_, (const T *)w_.z, &kc);
        if (rc) return rc;
        if (!std::isfinite(kc.r_p) || !std::isfinite(kc.r_d)) { status = SIPO_NUMERICAL; break; }
        // average: D_avg into tmp2, z_avg into Dn (Dn is free between iterations)
        rc = dose((const T *)y_avg, (T *)w_.tmp2);
        if (rc) return rc;
        double al1, aul2;
        rc = lambda_z(lu_avg, ll_avg, Dn, &al1, &aul2);
        if (rc) return rc;
        rc = kkt(y_avg, (const T *)w_.tmp2, hs_.u_avg, hs_.v_avg, lu_avg, ll_avg, Dn, &ka);
        if (rc) return rc;
        if (kc.rel() <= o_.tol) { status = SIPO_OPTIMAL; final_kkt = kc; break; }
        if (ka.rel() <= o_.tol) { status = SIPO_OPTIMAL; final_kkt = ka; use_avg_final = true; break; }
        bool infeasible = false;
        rc = farkas(o_.infeas_tol > 0 ? o_.infeas_tol : 1e-6, Dn, &infeasible);   // Dn is free here
        if (rc) return rc;
        if (infeasible) {
            status = SIPO_PRIMAL_INFEASIBLE;
            final_kkt = kc;
            break;
        }
        hipLaunchKernelGGL((k_copy<T>), dim3(gv_), dim3(kThreads), 0, s_, (T *)w_.lu_snap, (const T *)lu_, nv_);
        hipLaunchKernelGGL((k_copy<T>), dim3(gv_), dim3(kThreads), 0, s_, (T *)w_.ll_snap, (const T *)ll_, nv_);
        const double mc = kc.merit(), ma = ka.merit();
        const bool use_avg = ma < mc;
        const double mcand = std::min(ma, mc);
        const bool do_restart = mcand <= 0.2 * m_anchor || (mcand <= 0.8 * m_anchor && mcand > m_prev) ||
                                (double)(it - k_restart) >= 0.36 * (double)it;
        m_prev = mcand;
        if (!do_restart) continue;
        if (use_avg) {
            hipLaunchKernelGGL((k_copy<T>), dim3(gs_), dim3(kThreads), 0, s_, y_, (const T *)y_avg, ns_);
            hipLaunchKernelGGL((k_copy<T>), dim3(gv_), dim3(kThreads), 0, s_, lu_, (const T *)lu_avg, nv_);
            hipLaunchKernelGGL((k_copy<T>), dim3(gv_), dim3(kThreads), 0, s_, ll_, (const T *)ll_avg, nv_);
            hipLaunchKernelGGL((k_copy<T>), dim3(gv_), dim3(kThreads), 0, s_, D, (const T *)w_.tmp2, nv_);
            hs_.u = hs_.u_avg;
            hs_.v = hs_.v_avg;
        }
        // movement since the previous restart, in the scaled norms
        double dy2, dlu2, dll2;
        hipLaunchKernelGGL((k_wdist<T>), dim3(gs_), dim3(kThreads), 0, s_, (const T *)y_, (const T *)w_.y_anchor,
                           (const T *)w_.Tj, ns_, w_.partials);
        rc = sums(gs_, 1, &dy2);
        if (rc) return rc;
        hipLaunchKernelGGL((k_wdist<T>), dim3(gv_), dim3(kThreads), 0, s_, (const T *)lu_, (const T *)w_.lu_anchor,
                           (const T *)w_.s_up, nv_, w_.partials);
        rc = sums(gv_, 1, &dlu2);
        if (rc) return rc;
        hipLaunchKernelGGL((k_wdist<T>), dim3(gv_), dim3(kThreads), 0, s_, (const T *)ll_, (const T *)w_.ll_anchor,
                           (const T *)w_.s_lo, nv_, w_.partials);
        rc = sums(gv_, 1, &dll2);
        if (rc) return rc;
        const double du = hs_.u - anchor_u_, dv = hs_.v - anchor_v_;
        double dx2 = dy2 + (Tu_ > 0 ? du * du / Tu_ : 0.0) + (Tv_ > 0 ? dv * dv / Tv_ : 0.0);
        const double dx = std::sqrt(dx2), dl = std::sqrt(dlu2 + dll2);
        if (dx > 1e-10 && dl > 1e-10) omega = std::exp(0.5 * std::log(dl / dx) + 0.5 * std::log(omega));
        // new anchor / average start / z and lambda sums of the restart point
        hipLaunchKernelGGL((k_copy<T>), dim3(gs_), dim3(kThreads), 0, s_, (T *)w_.y_anchor, (const T *)y_, ns_);
        hipLaunchKernelGGL((k_copy<T>), dim3(gs_), dim3(kThreads), 0, s_, (T *)w_.y_avg, (const T *)y_, ns_);
        for (auto pr : {std::make_pair(w_.lu_anchor, (void *)lu_), std::make_pair(w_.ll_anchor, (void *)ll_),
                        std::make_pair(w_.lu_avg, (void *)lu_), std::make_pair(w_.ll_avg, (void *)ll_)})
            hipLaunchKernelGGL((k_copy<T>), dim3(gv_), dim3(kThreads), 0, s_, (T *)pr.first, (const T *)pr.second, nv_);
        double l1, ul2;
        rc = lambda_z(lu_, ll_, (T *)w_.z, &l1, &ul2);
        if (rc) return rc;
        hs_.sums[0] = l1;
        hs_.sums[1] = ul2;
        anchor_u_ = hs_.u;
        anchor_v_ = hs_.v;
        hs_.tau_fac = eta / omega;
        hs_.sig_fac = eta * omega;
        hs_.tau_u = eta * Tu_ / omega;
        hs_.tau_v = eta * Tv_ / omega;
        hs_.n_avg = 1.0;
        hs_.avg_w = 1.0;
        hs_.u_avg = hs_.u;
        hs_.v_avg = hs_.v;
        rc = put_scal();
        if (rc) return rc;
        hipLaunchKernelGGL(k_scalars_init, dim3(1), dim3(1), 0, s_, w_.scal, c_);
        m_anchor = use_avg ? ka.merit() : kc.merit();
        m_prev = 1e300;
        k_restart = it;
        ++restarts;
    }
    // ---------------- final point
    rc = get_scal();
    if (rc) return rc;
    double u = hs_.u, v = hs_.v;
    if (use_avg_final) {
        hipLaunchKernelGGL((k_copy<T>), dim3(gs_), dim3(kThreads), 0, s_, y_, (const T *)y_avg, ns_);
        hipLaunchKernelGGL((k_copy<T>), dim3(gv_), dim3(kThreads), 0, s_, lu_, (const T *)lu_avg, nv_);
        hipLaunchKernelGGL((k_copy<T>), dim3(gv_), dim3(kThreads), 0, s_, ll_, (const T *)ll_avg, nv_);
        hipLaunchKernelGGL((k_copy<T>), dim3(gv_), dim3(kThreads), 0, s_, D, (const T *)w_.tmp2, nv_);
        u = hs_.u_avg;
        v = hs_.v_avg;
    }
    if (status == SIPO_PRIMAL_INFEASIBLE) {
        // the certificate d = max(lambda - snapshot, 0) replaces lambda; the KKT fields keep the last iterate's
        hipLaunchKernelGGL((k_certificate<T>), dim3(gv_), dim3(kThreads), 0, s_, lu_, ll_, (const T *)w_.lu_snap,
                           (const T *)w_.ll_snap, lab_, nv_);
    } else if (status != SIPO_OPTIMAL) {
        hipLaunchKernelGGL((k_lambda_z<T>), dim3(gv_), dim3(kThreads), 0, s_, lu_, ll_, (T *)w_.z, lab_, hi_, c_, nv_,
                           w_.partials);
        rc = kkt(y_, D, u, v, lu_, ll_, (const T *)w_.z, &final_kkt);
        if (rc) return rc;
    }
    if (pb_.dose_out) {
        hipLaunchKernelGGL((k_copy<T>), dim3(gv_), dim3(kThreads), 0, s_, (T *)pb_.dose_out, (const T *)D, nv_);
    }
    SIPO_HIP(hipStreamSynchronize(s_));
    res->status = status;
    res->iters = it;
    res->restarts = restarts;
    res->primal_obj = final_kkt.p;
    res->dual_obj = final_kkt.d;
    res->rel_primal = final_kkt.eps_p;
    res->rel_dual = final_kkt.eps_d;
    res->rel_gap = final_kkt.eps_gap;
    res->u = u;
    res->v = v;
    res->tau = tau;
    res->sigma = sigma;
    res->omega = omega;
    res->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
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
    for (int i = 0; i < n; ++i) {
        Workspace w;
        layout(probs[i], &w, (char *)workspace);
        int rc = probs[i].plan->dtype == SIPO_F64
                     ? Solver<double>(probs[i], *opts, w, s).run(&results[i])
                     : Solver<float>(probs[i], *opts, w, s).run(&results[i]);
        if (rc) return rc;
    }
    return SIPO_OK;
}

}  // extern "C"
