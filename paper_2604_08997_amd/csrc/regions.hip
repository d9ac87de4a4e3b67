// Domain partition (Sec. 2.2, Fig. 2): gel / band / exterior labels and the
// active-ray mask.
//
// The band is "within Euclidean distance w of the gel" (plus the PSF's box
// support around the gel).  The squared distance to the nearest gel voxel is
// separable, d(x,y,z) = min_dz [dz^2 + min_dy [dy^2 + min_dx dx^2]], so three
// window passes of radius W = floor(w) give it exactly inside the window;
// values beyond w^2 saturate at 127 (w <= 11 keeps w^2 below that).  The top
// bit carries the box-dilation flag of the PSF support through the same
// passes.  All integer arithmetic: labels are bit-exact.
#include "sipo_internal.hpp"

namespace sipo {

constexpr uint8_t kInf = 127;

__device__ __forceinline__ bool in_vial(int c, int r, double h) {
    const double x = centre(c, h), y = centre(r, h);
    return fma(x, x, y * y) <= 1.0;
}

template <typename T>
__global__ void regions_pass_x(const T *__restrict__ f, uint8_t *__restrict__ out, int n, int nz, int W, int rx,
                               double h) {
    const size_t nvox = (size_t)nz * n * n;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nvox; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % n);
        const int r = (int)((i / n) % n);
        const size_t rowbase = i - c;
        int d = kInf;
        bool box = false;
        const int R = max(W, rx);
        for (int dx = -R; dx <= R; ++dx) {
            const int cc = c + dx;
            if (cc < 0 || cc >= n) continue;
            if (f[rowbase + cc] != (T)0 && in_vial(cc, r, h)) {
                if (abs(dx) <= W) d = min(d, dx * dx);
                if (abs(dx) <= rx) box = true;
            }
        }
        out[i] = (uint8_t)((box ? 0x80 : 0) | min(d, (int)kInf));
    }
}

// One pass along y (stride n) or z (stride n*n): min over |k| <= W of d + k^2, OR of the box flag over |k| <= rb.
__global__ void regions_pass_yz(const uint8_t *__restrict__ in, uint8_t *__restrict__ out, int n, int nz, int W, int rb,
                                int axis) {
    const size_t nvox = (size_t)nz * n * n;
    const size_t stride = axis == 1 ? (size_t)n : (size_t)n * n;
    const int len = axis == 1 ? n : nz;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nvox; i += (size_t)gridDim.x * blockDim.x) {
        const int pos = axis == 1 ? (int)((i / n) % n) : (int)(i / ((size_t)n * n));
        int d = kInf;
        bool box = false;
        const int R = max(W, rb);
        for (int k = -R; k <= R; ++k) {
            const int p = pos + k;
            if (p < 0 || p >= len) continue;
            const uint8_t v = in[(size_t)((long long)i + (long long)k * (long long)stride)];
            if (abs(k) <= W) d = min(d, (int)(v & 0x7f) + k * k);
            if (abs(k) <= rb && (v & 0x80)) box = true;
        }
        out[i] = (uint8_t)((box ? 0x80 : 0) | min(d, (int)kInf));
    }
}

template <typename T>
__global__ void regions_final(const T *__restrict__ f, const uint8_t *__restrict__ dist, uint8_t *__restrict__ lab,
                              int n, int nz, double w2, int band_free, double h) {
    const size_t nvox = (size_t)nz * n * n;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nvox; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % n);
        const int r = (int)((i / n) % n);
        uint8_t L = 0;
        if (in_vial(c, r, h)) {
            if (f[i] != (T)0) L = 2;
            else if (band_free) L = 1;
            else {
                const uint8_t v = dist[i];
                if ((v & 0x80) || (double)(v & 0x7f) <= w2) L = 1;
            }
        }
        lab[i] = L;
    }
}

template <typename T>
static int regions_impl(sipo_plan p, const void *f, double w, uint8_t *lab, uint8_t *scratch, hipStream_t s) {
    const int n = p->n, nz = p->nz;
    const double h = 2.0 / n;
    const size_t nvox = p->vol_elems();
    const int threads = 256;
    const int blocks = (int)std::min<size_t>((nvox + threads - 1) / threads, 65536);
    if (w < 0) {
        hipLaunchKernelGGL((regions_final<T>), dim3(blocks), dim3(threads), 0, s, (const T *)f, scratch, lab, n, nz,
                           0.0, 1, h);
        SIPO_LAUNCHED("regions_final");
        return SIPO_OK;
    }
    const int W = (int)std::floor(w);
    const int rx = p->has_psf ? p->taps_f.rx : 0, ry = p->has_psf ? p->taps_f.ry : 0, rz = p->has_psf ? p->taps_f.rz : 0;
    hipLaunchKernelGGL((regions_pass_x<T>), dim3(blocks), dim3(threads), 0, s, (const T *)f, lab, n, nz, W, rx, h);
    SIPO_LAUNCHED("regions_pass_x");
    hipLaunchKernelGGL(regions_pass_yz, dim3(blocks), dim3(threads), 0, s, lab, scratch, n, nz, W, ry, 1);
    SIPO_LAUNCHED("regions_pass_y");
    hipLaunchKernelGGL(regions_pass_yz, dim3(blocks), dim3(threads), 0, s, scratch, lab, n, nz, W, rz, 2);
    SIPO_LAUNCHED("regions_pass_z");
    // final labels: read the distances from lab into scratch first is unnecessary; regions_final
    // reads dist and writes lab at the same index only, so in-place use of one buffer is safe.
    hipLaunchKernelGGL((regions_final<T>), dim3(blocks), dim3(threads), 0, s, (const T *)f, lab, lab, n, nz, w * w, 0,
                       h);
    SIPO_LAUNCHED("regions_final");
    return SIPO_OK;
}

// ---------------------------------------------------------- active rays
template <typename T>
struct MaxBits;
template <>
struct MaxBits<float> {
    using U = unsigned int;
    static __device__ U bits(float v) { return __float_as_uint(v); }
    static __device__ float val(U b) { return __uint_as_float(b); }
};
template <>
struct MaxBits<double> {
    using U = unsigned long long;
    static __device__ U bits(double v) { return (U)__double_as_longlong(v); }
    static __device__ double val(U b) { return __longlong_as_double((long long)b); }
};

template <typename T>
__global__ void zero_bits(typename MaxBits<T>::U *m) { *m = 0; }

template <typename T>
__global__ void max_nonneg(const T *__restrict__ v, size_t count, typename MaxBits<T>::U *m) {
    using U = typename MaxBits<T>::U;
    __shared__ U part[256];
    U best = 0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
        const T x = v[i];
        const U b = MaxBits<T>::bits(x > (T)0 ? x : (T)0);   // non-negative: bit order == value order
        best = b > best ? b : best;
    }
    part[threadIdx.x] = best;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) part[threadIdx.x] = max(part[threadIdx.x], part[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(m, part[0]);
}

template <typename T>
__global__ void threshold_act(const T *__restrict__ v, size_t count, const typename MaxBits<T>::U *m, T rel,
                              uint8_t *__restrict__ act) {
    const T thr = rel * MaxBits<T>::val(*m);
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        act[i] = (v[i] > thr && thr > (T)0) ? 1 : 0;
}

template <typename T>
static int act_impl(sipo_plan p, const void *f, void *pf, uint8_t *act, hipStream_t s) {
    int rc = check_plan_ws(p);
    if (!rc) rc = launch_project(p, f, pf, 0, s);
    if (rc) return rc;
    using U = typename MaxBits<T>::U;
    U *m = (U *)p->ws_red();
    const size_t count = p->sino_elems();
    const int blocks = (int)std::min<size_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL((zero_bits<T>), dim3(1), dim3(1), 0, s, m);
    hipLaunchKernelGGL((max_nonneg<T>), dim3(blocks), dim3(256), 0, s, (const T *)pf, count, m);
    hipLaunchKernelGGL((threshold_act<T>), dim3(blocks), dim3(256), 0, s, (const T *)pf, count, (const U *)m, (T)1e-6,
                       act);
    SIPO_LAUNCHED("active_rays");
    return SIPO_OK;
}

}  // namespace sipo

using namespace sipo;

extern "C" {

int sipo_regions(sipo_plan plan, const void *f_target, double band_width, uint8_t *labels, uint8_t *scratch,
                 void *stream) {
    int rc = check_plan(plan);
    if (rc) return rc;
    SIPO_REQUIRE(f_target && labels && scratch, "f_target, labels or scratch is NULL");
    SIPO_REQUIRE((void *)labels != (void *)scratch, "labels and scratch must differ");
    SIPO_REQUIRE(std::isfinite(band_width) || band_width < 0, "band_width must be finite or negative");
    SIPO_REQUIRE(band_width < 0 || band_width <= SIPO_MAX_BAND_WIDTH, "band_width %g exceeds %g (use < 0 for band-free)",
                 band_width, SIPO_MAX_BAND_WIDTH);
    return plan->dtype == SIPO_F64 ? regions_impl<double>(plan, f_target, band_width, labels, scratch, (hipStream_t)stream)
                                   : regions_impl<float>(plan, f_target, band_width, labels, scratch, (hipStream_t)stream);
}

int sipo_active_rays(sipo_plan plan, const void *f_target, void *scratch_sino, uint8_t *act, void *stream) {
    int rc = check_plan(plan);
    if (rc) return rc;
    SIPO_REQUIRE(f_target && scratch_sino && act, "f_target, scratch_sino or act is NULL");
    return plan->dtype == SIPO_F64 ? act_impl<double>(plan, f_target, scratch_sino, act, (hipStream_t)stream)
                                   : act_impl<float>(plan, f_target, scratch_sino, act, (hipStream_t)stream);
}

}  // extern "C"
