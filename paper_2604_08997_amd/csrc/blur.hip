// Object-space PSF K (Eq. 1-3): separable convolution with zero boundary,
// fused into one pass over HBM.
//
// A workgroup owns a 64 x 16 (x, y) tile and a chunk of slices.  It streams
// the slices in z order: each slice tile (with its x/y halo) is staged in LDS,
// blurred along x and then y, and the xy-blurred values of a thread's four
// columns are pushed through a register ring of 2 rz + 1 slices; when the
// ring is full the z taps produce one output slice.  Every input slice is
// read from HBM once per tile (plus halos) and every output written once.
#include "sipo_internal.hpp"

namespace sipo {

constexpr int kBTX = 64, kBTY = 16, kBRows = 4;   // tile and rows per thread (256 threads)

template <typename T, int RZ>
__global__ void __launch_bounds__(256) blur_kernel(const T *__restrict__ in, T *__restrict__ out, int n, int nz,
                                                   Taps<T> tp, int zchunk) {
    __shared__ T raw[(kBTY + 2 * kMaxR) * (kBTX + 2 * kMaxR)];
    __shared__ T xb[(kBTY + 2 * kMaxR) * kBTX];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = ty * kBTX + tx;
    const int x0 = blockIdx.x * kBTX, y0 = blockIdx.y * kBTY;
    const int z0 = blockIdx.z * zchunk;
    const int zend = min(nz, z0 + zchunk);
    const int rx = tp.rx, ry = tp.ry;
    const int RW = kBTX + 2 * rx, RH = kBTY + 2 * ry;
    const size_t plane = (size_t)n * n;
    T ring[kBRows][2 * RZ + 1];
#pragma unroll
    for (int j = 0; j < kBRows; ++j)
#pragma unroll
        for (int m = 0; m < 2 * RZ + 1; ++m) ring[j][m] = (T)0;

    for (int zi = z0 - RZ; zi < zend + RZ; ++zi) {
        T v[kBRows];
        if (zi >= 0 && zi < nz) {
            const T *src = in + (size_t)zi * plane;
            for (int e = tid; e < RW * RH; e += 256) {
                const int ly = e / RW, lx = e - ly * RW;
                const int gy = y0 - ry + ly, gx = x0 - rx + lx;
                raw[ly * (kBTX + 2 * kMaxR) + lx] =
                    (gx >= 0 && gx < n && gy >= 0 && gy < n) ? src[(size_t)gy * n + gx] : (T)0;
            }
            __syncthreads();
            for (int e = tid; e < RH * kBTX; e += 256) {
                const int ly = e / kBTX, lx = e - ly * kBTX;
                const T *rr = raw + ly * (kBTX + 2 * kMaxR) + lx;
                T s = (T)0;
                for (int k = 0; k <= 2 * rx; ++k) s = fma(tp.kx[k], rr[k], s);
                xb[ly * kBTX + lx] = s;
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kBRows; ++j) {
                const int ly = ty + 4 * j;
                T s = (T)0;
                for (int k = 0; k <= 2 * ry; ++k) s = fma(tp.ky[k], xb[(ly + k) * kBTX + tx], s);
                v[j] = s;
            }
        } else {
#pragma unroll
            for (int j = 0; j < kBRows; ++j) v[j] = (T)0;
        }
#pragma unroll
        for (int j = 0; j < kBRows; ++j) {
#pragma unroll
            for (int m = 0; m < 2 * RZ; ++m) ring[j][m] = ring[j][m + 1];
            ring[j][2 * RZ] = v[j];
        }
        const int zo = zi - RZ;
        if (zo >= z0 && zo < zend) {
            const int gx = x0 + tx;
#pragma unroll
            for (int j = 0; j < kBRows; ++j) {
                const int gy = y0 + ty + 4 * j;
                T s = (T)0;
#pragma unroll
                for (int m = 0; m < 2 * RZ + 1; ++m) s = fma(tp.kz[m], ring[j][m], s);
                if (gx < n && gy < n) out[(size_t)zo * plane + (size_t)gy * n + gx] = s;
            }
        }
    }
}

template <typename T, int RZ>
static void launch_rz(const Taps<T> &tp, const void *in, void *out, int n, int nz, hipStream_t s) {
    const int zchunk = nz <= 32 ? nz : 32;
    const dim3 grid((n + kBTX - 1) / kBTX, (n + kBTY - 1) / kBTY, (nz + zchunk - 1) / zchunk);
    hipLaunchKernelGGL((blur_kernel<T, RZ>), grid, dim3(kBTX, 4), 0, s, (const T *)in, (T *)out, n, nz, tp, zchunk);
}

template <typename T>
static int blur_dispatch(sipo_plan p, const Taps<T> &tp, const void *in, void *out, hipStream_t s) {
    switch (tp.rz) {
        case 0: launch_rz<T, 0>(tp, in, out, p->n, p->nz, s); break;
        case 1: launch_rz<T, 1>(tp, in, out, p->n, p->nz, s); break;
        case 2: launch_rz<T, 2>(tp, in, out, p->n, p->nz, s); break;
        case 3: launch_rz<T, 3>(tp, in, out, p->n, p->nz, s); break;
        case 4: launch_rz<T, 4>(tp, in, out, p->n, p->nz, s); break;
        case 5: launch_rz<T, 5>(tp, in, out, p->n, p->nz, s); break;
        case 6: launch_rz<T, 6>(tp, in, out, p->n, p->nz, s); break;
        case 7: launch_rz<T, 7>(tp, in, out, p->n, p->nz, s); break;
        case 8: launch_rz<T, 8>(tp, in, out, p->n, p->nz, s); break;
        default: return fail(SIPO_E_UNSUPPORTED, "PSF z radius %d > %d", tp.rz, kMaxR);
    }
    SIPO_LAUNCHED("blur_kernel");
    return SIPO_OK;
}

int launch_blur(sipo_plan p, const void *in, void *out, hipStream_t s) {
    if (!p->has_psf) {
        SIPO_HIP(hipMemcpyAsync(out, in, p->vol_elems() * p->elem_bytes(), hipMemcpyDeviceToDevice, s));
        return SIPO_OK;
    }
    return p->dtype == SIPO_F64 ? blur_dispatch<double>(p, p->taps_d, in, out, s)
                                : blur_dispatch<float>(p, p->taps_f, in, out, s);
}

}  // namespace sipo
