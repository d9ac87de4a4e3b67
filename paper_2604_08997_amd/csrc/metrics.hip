// Material response M / M^-1 (Eq. 4-5), scale-invariant metrics (Eq. 6-8, 46)
// and post-scaling (Eq. 25-28) of a normalised dose on the device.
//
// Each metric pass is one grid-stride kernel that leaves, per workgroup, eight
// FP64 fields (maxima, or sums) in the plan's workspace, finished by one block in
// a fixed order.  The response-domain calibration (Eq. 28) is a 1-D search on
// the host over alpha, each step one device reduction of
// sum_gel w (M(alpha D) - m_T)^2: a log-spaced scan around the dose-domain
// alpha_f followed by a golden-section refinement of the best bracket.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "sipo_internal.hpp"

namespace sipo {

constexpr int kMT = 256, kMF = 8, kMBlocks = 1024;
// device scratch of one evaluation: kMBlocks rows of kMF partials, then the kMF results
constexpr size_t kEvalScratchBytes = sizeof(double) * (size_t)(kMBlocks + 1) * kMF;
static_assert(kEvalScratchBytes <= kPlanRedBytes, "plan reduction area too small for the metric partials");

__device__ __forceinline__ double resp(const sipo_resin &r, double f) {
    return r.alpha + (r.k - r.alpha) / pow(1.0 + exp(-r.beta * (f - r.f0)), 1.0 / r.gamma);
}
__device__ __forceinline__ double resp_inv(const sipo_resin &r, double m) {
    return r.f0 - log(pow((r.k - r.alpha) / (m - r.alpha), r.gamma) - 1.0) / r.beta;
}

template <typename T>
__global__ void k_response(const T *in, T *out, size_t n, sipo_resin r, int inverse) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const double v = (double)in[i];
        out[i] = (T)(inverse ? resp_inv(r, v) : resp(r, v));
    }
}

// Per-field combination: bit k of max_mask set -> maximum, else sum.
__device__ __forceinline__ double comb(double a, double b, bool mx) { return mx ? fmax(a, b) : a + b; }

template <unsigned max_mask>
__device__ void block_store(double (&v)[kMF], double *partials) {
    __shared__ double red[kMT / 64][kMF];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kMF; ++k) {
        double x = v[k];
        for (int o = 32; o > 0; o >>= 1) x = comb(x, __shfl_down(x, o, 64), (max_mask >> k) & 1);
        if (lane == 0) red[w][k] = x;
    }
    __syncthreads();
    if (threadIdx.x < kMF) {
        const bool mx = (max_mask >> threadIdx.x) & 1;
        double x = red[0][threadIdx.x];
        for (int i = 1; i < kMT / 64; ++i) x = comb(x, red[i][threadIdx.x], mx);
        partials[blockIdx.x * kMF + threadIdx.x] = x;
    }
}

template <unsigned max_mask>
__global__ void __launch_bounds__(kMT) k_mfinish(const double *partials, int nblocks, double *out) {
    const int k = threadIdx.x;
    if (k >= kMF) return;
    const bool mx = (max_mask >> k) & 1;
    double x = partials[k];
    for (int b = 1; b < nblocks; ++b) x = comb(x, partials[b * kMF + k], mx);
    out[k] = x;
}

// Pass 1: [0] max_gel r, [1] max_gel -r, [2] max_band D, [3] max_gel -D  (r = D / f~_T),
//         [4] sum_gel w D f_T, [5] sum_gel w D^2, [6] |gel|, [7] |band|
constexpr unsigned kMask1 = 0x0Fu;
template <typename T>
__global__ void __launch_bounds__(kMT) k_eval1(const T *D, const uint8_t *lab, const T *ftn, double fts, double fcrit,
                                                const T *w, size_t n, double *partials) {
    const double ninf = -INFINITY;
    double v[kMF] = {ninf, ninf, ninf, ninf, 0, 0, 0, 0};
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const uint8_t L = lab[i];
        if (L == 0) continue;
        const double d = (double)D[i];
        if (L == 2) {
            const double ft = ftn ? (double)ftn[i] : fts;
            const double r = d / ft, wi = w ? (double)w[i] : 1.0;
            v[0] = fmax(v[0], r);
            v[1] = fmax(v[1], -r);
            v[3] = fmax(v[3], -d);
            v[4] += wi * d * (fcrit * ft);
            v[5] += wi * d * d;
            v[6] += 1.0;
        } else {
            v[2] = fmax(v[2], d);
            v[7] += 1.0;
        }
    }
    block_store<kMask1>(v, partials);
}

// Pass 2 at alpha: [0] sum_gel w (M(alpha D) - m_T)^2, [1] max_gel M/m_T, [2] max_gel -(M/m_T),
//                  [3] max_gel -M, [4] max_band M
constexpr unsigned kMask2 = 0x1Eu;
template <typename T>
__global__ void __launch_bounds__(kMT) k_eval2(const T *D, const uint8_t *lab, const T *mt, double mts, const T *w,
                                                double alpha, sipo_resin r, size_t n, double *partials) {
    const double ninf = -INFINITY;
    double v[kMF] = {0, ninf, ninf, ninf, ninf, 0, 0, 0};
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const uint8_t L = lab[i];
        if (L == 0) continue;
        const double m = resp(r, alpha * (double)D[i]);
        if (L == 2) {
            const double t = mt ? (double)mt[i] : mts, wi = w ? (double)w[i] : 1.0;
            v[0] += wi * (m - t) * (m - t);
            v[1] = fmax(v[1], m / t);
            v[2] = fmax(v[2], -(m / t));
            v[3] = fmax(v[3], -m);
        } else {
            v[4] = fmax(v[4], m);
        }
    }
    block_store<kMask2>(v, partials);
}

static int check_resin(const sipo_resin *r) {
    SIPO_REQUIRE(r != nullptr, "resin is NULL");
    SIPO_REQUIRE(std::isfinite(r->alpha) && std::isfinite(r->k) && std::isfinite(r->beta) && std::isfinite(r->gamma) &&
                     std::isfinite(r->f0),
                 "resin constants must be finite");
    SIPO_REQUIRE(r->k != r->alpha && r->beta != 0.0 && r->gamma > 0.0, "resin needs k != alpha, beta != 0, gamma > 0");
    return SIPO_OK;
}

template <typename T>
class Evaluator {
  public:
    // scratch: kEvalScratchBytes of device memory for the per-workgroup partials and the result
    Evaluator(sipo_plan p, const T *D, const uint8_t *lab, const T *w, double *scratch, hipStream_t s)
        : p_(p), D_(D), lab_(lab), w_(w), s_(s), n_(p->vol_elems()) {
        nb_ = (int)std::max<size_t>(1, std::min<size_t>((n_ + 4 * kMT - 1) / (4 * kMT), kMBlocks));
        partials_ = scratch;
        out_ = partials_ + (size_t)kMBlocks * kMF;
    }
    int pass1(const T *ftn, double fts, double fcrit, double *h) {
        hipLaunchKernelGGL((k_eval1<T>), dim3(nb_), dim3(kMT), 0, s_, D_, lab_, ftn, fts, fcrit, w_, n_, partials_);
        hipLaunchKernelGGL(k_mfinish<kMask1>, dim3(1), dim3(kMT), 0, s_, partials_, nb_, out_);
        return fetch(h);
    }
    int pass2(const T *mt, double mts, double alpha, const sipo_resin &r, double *h) {
        hipLaunchKernelGGL((k_eval2<T>), dim3(nb_), dim3(kMT), 0, s_, D_, lab_, mt, mts, w_, alpha, r, n_, partials_);
        hipLaunchKernelGGL(k_mfinish<kMask2>, dim3(1), dim3(kMT), 0, s_, partials_, nb_, out_);
        return fetch(h);
    }

  private:
    int fetch(double *h) {
        SIPO_LAUNCHED("metrics");
        SIPO_HIP(hipMemcpyAsync(h, out_, sizeof(double) * kMF, hipMemcpyDeviceToHost, s_));
        SIPO_HIP(hipStreamSynchronize(s_));
        return SIPO_OK;
    }
    sipo_plan p_;
    const T *D_;
    const uint8_t *lab_;
    const T *w_;
    hipStream_t s_;
    size_t n_;
    int nb_;
    double *partials_, *out_;
};

template <typename T>
static int evaluate(sipo_plan p, const void *dose, const uint8_t *labels, const void *ftn, double fts, double fcrit,
                    const void *weights, const sipo_resin *resin, const void *mt, double mts, sipo_metrics *o,
                    double *scratch, hipStream_t s) {
    Evaluator<T> ev(p, (const T *)dose, labels, (const T *)weights, scratch, s);
    double h[kMF];
    int rc = ev.pass1((const T *)ftn, fts, fcrit, h);
    if (rc) return rc;
    const double nan = std::nan("");
    o->n_gel = (int64_t)h[6];
    o->n_band = (int64_t)h[7];
    o->gel_ratio_max = o->n_gel ? h[0] : nan;
    o->gel_ratio_min = o->n_gel ? -h[1] : nan;
    o->gel_min = o->n_gel ? -h[3] : nan;
    o->band_max = o->n_band ? h[2] : nan;
    const double lo = o->gel_ratio_min;
    o->dtvr = lo > 0 ? o->gel_ratio_max / lo : INFINITY;
    o->dsr = !o->n_band ? nan : (lo > 0 ? o->band_max / lo : INFINITY);
    o->psr_f = !o->n_band ? nan : (o->band_max > 0 ? o->gel_min / o->band_max : INFINITY);
    o->alpha_f = h[5] > 0 ? h[4] / h[5] : nan;
    o->alpha_m = o->psr_m = o->dtvr_m = nan;
    if (!resin) return SIPO_OK;
    // Eq. 28: scan log(alpha) over [a0 / 100, a0 * 100] around the dose-domain alpha, then golden section
    const double a0 = (std::isfinite(o->alpha_f) && o->alpha_f > 0) ? o->alpha_f : 1.0;
    constexpr int kScan = 41;
    const double L0 = std::log(a0) - std::log(100.0), L1 = std::log(a0) + std::log(100.0);
    auto phi = [&](double la, double *hh) { return ev.pass2((const T *)mt, mts, std::exp(la), *resin, hh); };
    std::vector<double> f(kScan);
    int best = 0;
    for (int i = 0; i < kScan; ++i) {
        rc = phi(L0 + (L1 - L0) * i / (kScan - 1), h);
        if (rc) return rc;
        f[i] = std::isfinite(h[0]) ? h[0] : INFINITY;
        if (f[i] < f[best]) best = i;
    }
    double a = L0 + (L1 - L0) * std::max(best - 1, 0) / (kScan - 1);
    double b = L0 + (L1 - L0) * std::min(best + 1, kScan - 1) / (kScan - 1);
    const double g = 0.5 * (std::sqrt(5.0) - 1.0);
    double c = b - g * (b - a), d = a + g * (b - a), fc, fd;
    rc = phi(c, h); if (rc) return rc; fc = h[0];
    rc = phi(d, h); if (rc) return rc; fd = h[0];
    for (int it = 0; it < 80 && (b - a) > 1e-13 * (1.0 + std::fabs(a)); ++it) {
        if (fc <= fd) { b = d; d = c; fd = fc; c = b - g * (b - a); rc = phi(c, h); fc = h[0]; }
        else { a = c; c = d; fc = fd; d = a + g * (b - a); rc = phi(d, h); fd = h[0]; }
        if (rc) return rc;
    }
    o->alpha_m = std::exp(0.5 * (a + b));
    rc = ev.pass2((const T *)mt, mts, o->alpha_m, *resin, h);
    if (rc) return rc;
    const double mlo = -h[2];
    o->dtvr_m = o->n_gel ? (mlo > 0 ? h[1] / mlo : INFINITY) : nan;
    o->psr_m = !o->n_band ? nan : (h[4] > 0 ? -h[3] / h[4] : INFINITY);
    return SIPO_OK;
}

// Argument checks shared by sipo_evaluate and sipo_evaluate_noalloc.
static int check_eval_args(sipo_plan plan, const void *dose, const uint8_t *labels, const void *f_target_norm,
                           double f_t_scalar, double f_crit, const sipo_resin *resin, const void *m_target,
                           double m_t_scalar, const sipo_metrics *out) {
    int rc = check_plan(plan);
    if (rc) return rc;
    SIPO_REQUIRE(dose && labels && out, "dose, labels or out is NULL");
    SIPO_REQUIRE(f_target_norm || (std::isfinite(f_t_scalar) && f_t_scalar > 0), "f~_T scalar must be > 0");
    SIPO_REQUIRE(std::isfinite(f_crit) && f_crit > 0, "f_crit must be finite and > 0");
    if (resin) {
        rc = check_resin(resin);
        if (rc) return rc;
        SIPO_REQUIRE(m_target || std::isfinite(m_t_scalar), "m_T scalar must be finite");
    }
    return SIPO_OK;
}

static int run_evaluate(sipo_plan plan, const void *dose, const uint8_t *labels, const void *ftn, double fts,
                        double fcrit, const void *weights, const sipo_resin *resin, const void *mt, double mts,
                        sipo_metrics *out, double *scratch, hipStream_t s) {
    return plan->dtype == SIPO_F64
               ? evaluate<double>(plan, dose, labels, ftn, fts, fcrit, weights, resin, mt, mts, out, scratch, s)
               : evaluate<float>(plan, dose, labels, ftn, fts, fcrit, weights, resin, mt, mts, out, scratch, s);
}

// ------------------------------------------------- allocation-free evaluation
// Scratch of sipo_evaluate_noalloc: a file-scope device array.  Every GPU that loads the library
// holds its own copy until the process ends.  On the host the array's name is only a stand-in
// symbol, never a device address: the address of the current device's copy is looked up once per
// device with hipGetSymbolAddress and kept in g_noalloc_ptr, and only that pointer reaches kernels.
constexpr size_t kNoAllocScratchBytes = kEvalScratchBytes;   // 65,600 bytes
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];
constexpr int kMaxDevices = 64;
static std::mutex g_noalloc_mu;
static double *g_noalloc_ptr[kMaxDevices] = {};

static int noalloc_scratch(int dev, double **out) {
    *out = nullptr;
    SIPO_REQUIRE(dev >= 0 && dev < kMaxDevices, "device %d outside the supported range [0, %d)", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr)
            return fail(SIPO_E_DEVICE, "hipGetSymbolAddress of the evaluation scratch failed on device %d: %s", dev,
                        hipGetErrorString(e));
        g_noalloc_ptr[dev] = (double *)ptr;
    }
    *out = g_noalloc_ptr[dev];
    return SIPO_OK;
}

}  // namespace sipo

using namespace sipo;

extern "C" {

int sipo_response(sipo_plan plan, const sipo_resin *resin, const void *in, void *out, int inverse, void *stream) {
    int rc = check_plan(plan);
    if (!rc) rc = check_resin(resin);
    if (rc) return rc;
    SIPO_REQUIRE(in && out, "in or out is NULL");
    const size_t n = plan->vol_elems();
    const int grid = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipStream_t s = (hipStream_t)stream;
    if (plan->dtype == SIPO_F64)
        hipLaunchKernelGGL((k_response<double>), dim3(grid), dim3(256), 0, s, (const double *)in, (double *)out, n,
                           *resin, inverse);
    else
        hipLaunchKernelGGL((k_response<float>), dim3(grid), dim3(256), 0, s, (const float *)in, (float *)out, n,
                           *resin, inverse);
    SIPO_LAUNCHED("k_response");
    return SIPO_OK;
}

int sipo_evaluate(sipo_plan plan, const void *dose, const uint8_t *labels, const void *f_target_norm,
                  double f_t_scalar, double f_crit, const void *weights, const sipo_resin *resin,
                  const void *m_target, double m_t_scalar, sipo_metrics *out, void *stream) {
    int rc = check_eval_args(plan, dose, labels, f_target_norm, f_t_scalar, f_crit, resin, m_target, m_t_scalar, out);
    if (!rc) rc = check_plan_ws(plan);
    if (rc) return rc;
    return run_evaluate(plan, dose, labels, f_target_norm, f_t_scalar, f_crit, weights, resin, m_target, m_t_scalar,
                        out, (double *)plan->ws_red(), (hipStream_t)stream);
}

int sipo_evaluate_noalloc(sipo_plan plan, const void *dose, const uint8_t *labels, const void *f_target_norm,
                          double f_t_scalar, double f_crit, const void *weights, const sipo_resin *resin,
                          const void *m_target, double m_t_scalar, sipo_metrics *out, void *stream) {
    int rc = check_eval_args(plan, dose, labels, f_target_norm, f_t_scalar, f_crit, resin, m_target, m_t_scalar, out);
    if (rc) return rc;
    // the reduction runs at most kMBlocks workgroups whatever the volume size, so its partials and
    // result always fit the array; the test stays in case either constant changes
    const size_t blocks = std::max<size_t>(1, std::min<size_t>((plan->vol_elems() + 4 * kMT - 1) / (4 * kMT), kMBlocks));
    const size_t need = sizeof(double) * (size_t)kMF * (kMBlocks + 1);
    SIPO_REQUIRE(blocks <= (size_t)kMBlocks && need <= kNoAllocScratchBytes,
                 "evaluation needs %zu bytes of scratch, above the %zu-byte array", need, kNoAllocScratchBytes);
    double *ptr = nullptr;
    rc = noalloc_scratch(plan->device, &ptr);
    if (rc) return rc;
    return run_evaluate(plan, dose, labels, f_target_norm, f_t_scalar, f_crit, weights, resin, m_target, m_t_scalar,
                        out, ptr, (hipStream_t)stream);
}

}  // extern "C"
