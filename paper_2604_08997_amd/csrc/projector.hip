// Backprojector P^T and projector P (Eq. 2-3): gathers in both directions.
//
// P^T: one thread per voxel column (x, y) and a chunk of ZC slices; the
//      per-view taps are computed once and reused for every slice of the
//      chunk, and the two sinogram samples of each tap pair are gathered.
// P:   one thread per detector bin and view and a chunk of ZC slices; the
//      ray is walked along its major axis and, per step, the few voxels
//      whose taps can reach the bin are tested with the same tap function
//      as P^T, which makes P the exact transpose of P^T.
#include "sipo_internal.hpp"

namespace sipo {

template <typename T, int ZC>
__global__ void __launch_bounds__(256) backproject_kernel(const T *__restrict__ sino, T *__restrict__ vol, int n,
                                                          int nz, int n_angles, int nb,
                                                          const double2 *__restrict__ trig, double h,
                                                          double inv_ds, T atten, int accumulate) {
    const int c = blockIdx.x * 64 + threadIdx.x;
    const int r = blockIdx.y * 4 + threadIdx.y;
    const int z0 = blockIdx.z * ZC;
    if (c >= n || r >= n) return;
    const double x = centre(c, h), y = centre(r, h);
    T acc[ZC];
#pragma unroll
    for (int k = 0; k < ZC; ++k) acc[k] = (T)0;
    const int zc = min(ZC, nz - z0);
    if (fma(x, x, y * y) <= 1.0) {
        for (int a = 0; a < n_angles; ++a) {
            const double2 tr = trig[a];
            T w0, w1;
            const int b = taps<T>(x, y, tr.x, tr.y, inv_ds, atten, w0, w1);
            const bool ok0 = b >= 0 && b < nb;
            const bool ok1 = b + 1 >= 0 && b + 1 < nb;
            const T *row = sino + ((size_t)a * nz + z0) * nb;
#pragma unroll
            for (int k = 0; k < ZC; ++k) {
                if (k < zc) {
                    const T s0 = ok0 ? row[(size_t)k * nb + b] : (T)0;
                    const T s1 = ok1 ? row[(size_t)k * nb + b + 1] : (T)0;
                    acc[k] = fma(w0, s0, acc[k]);
                    acc[k] = fma(w1, s1, acc[k]);
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < ZC; ++k) {
        if (k < zc) {
            const size_t idx = ((size_t)(z0 + k) * n + r) * n + c;
            vol[idx] = accumulate ? vol[idx] + acc[k] : acc[k];
        }
    }
}

template <typename T, int ZC>
__global__ void __launch_bounds__(256) project_kernel(const T *__restrict__ vol, T *__restrict__ sino, int n,
                                                      int nz, int n_angles, int nb,
                                                      const double2 *__restrict__ trig, double h,
                                                      double inv_ds, T atten, int accumulate) {
    const int b = blockIdx.x * 64 + threadIdx.x;
    const int a = blockIdx.y * 4 + threadIdx.y;
    const int z0 = blockIdx.z * ZC;
    if (b >= nb || a >= n_angles) return;
    const double2 tr = trig[a];
    const double sn = tr.x, cs = tr.y;
    T acc[ZC];
#pragma unroll
    for (int k = 0; k < ZC; ++k) acc[k] = (T)0;
    const int zc = min(ZC, nz - z0);
    const bool xmajor = fabs(cs) >= fabs(sn);
    // u along the minor axis: u(i_major, j_minor) ~ U(i_major) + j_minor * du
    const double du = (xmajor ? cs : -sn) * h * inv_ds;
    const double lo_t = (double)b - 1.0, hi_t = (double)b + 1.0;
    const double c0 = centre(0, h);
    for (int i = 0; i < n; ++i) {
        const double pm = centre(i, h);  // coordinate along the major axis
        // detector coordinate at minor index 0
        const double s0 = xmajor ? fma(-pm, sn, c0 * cs) : fma(-c0, sn, pm * cs);
        const double U = fma(s0 + 1.0, inv_ds, -0.5);
        double j1 = (lo_t - U) / du, j2 = (hi_t - U) / du;
        if (j1 > j2) { const double tmp = j1; j1 = j2; j2 = tmp; }
        int jlo = (int)floor(j1) - 1, jhi = (int)ceil(j2) + 1;
        jlo = max(jlo, 0);
        jhi = min(jhi, n - 1);
        for (int j = jlo; j <= jhi; ++j) {
            const int c = xmajor ? i : j;
            const int r = xmajor ? j : i;
            const double x = centre(c, h), y = centre(r, h);
            if (fma(x, x, y * y) > 1.0) continue;
            T w0, w1;
            const int bv = taps<T>(x, y, sn, cs, inv_ds, atten, w0, w1);
            T w;
            if (bv == b) w = w0;
            else if (bv == b - 1) w = w1;
            else continue;
            const T *src = vol + (size_t)r * n + c;
#pragma unroll
            for (int k = 0; k < ZC; ++k)
                if (k < zc) acc[k] = fma(w, src[(size_t)(z0 + k) * n * n], acc[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < ZC; ++k) {
        if (k < zc) {
            const size_t idx = ((size_t)a * nz + z0 + k) * nb + b;
            sino[idx] = accumulate ? sino[idx] + acc[k] : acc[k];
        }
    }
}

template <typename T>
static int bp_dispatch(sipo_plan p, const void *sino, void *vol, int accumulate, hipStream_t s) {
    const double h = 2.0 / p->n, inv_ds = 0.5 * p->n_bins;
    const dim3 block(64, 4);
    if (p->nz == 1) {
        const dim3 grid((p->n + 63) / 64, (p->n + 3) / 4, 1);
        hipLaunchKernelGGL((backproject_kernel<T, 1>), grid, block, 0, s, (const T *)sino, (T *)vol, p->n, p->nz,
                           p->n_angles, p->n_bins, p->d_trig, h, inv_ds, (T)p->atten, accumulate);
    } else {
        constexpr int ZC = 8;
        const dim3 grid((p->n + 63) / 64, (p->n + 3) / 4, (p->nz + ZC - 1) / ZC);
        hipLaunchKernelGGL((backproject_kernel<T, ZC>), grid, block, 0, s, (const T *)sino, (T *)vol, p->n, p->nz,
                           p->n_angles, p->n_bins, p->d_trig, h, inv_ds, (T)p->atten, accumulate);
    }
    SIPO_LAUNCHED("backproject_kernel");
    return SIPO_OK;
}

template <typename T>
static int fp_dispatch(sipo_plan p, const void *vol, void *sino, int accumulate, hipStream_t s) {
    const double h = 2.0 / p->n, inv_ds = 0.5 * p->n_bins;
    const dim3 block(64, 4);
    if (p->nz == 1) {
        const dim3 grid((p->n_bins + 63) / 64, (p->n_angles + 3) / 4, 1);
        hipLaunchKernelGGL((project_kernel<T, 1>), grid, block, 0, s, (const T *)vol, (T *)sino, p->n, p->nz,
                           p->n_angles, p->n_bins, p->d_trig, h, inv_ds, (T)p->atten, accumulate);
    } else {
        constexpr int ZC = 8;
        const dim3 grid((p->n_bins + 63) / 64, (p->n_angles + 3) / 4, (p->nz + ZC - 1) / ZC);
        hipLaunchKernelGGL((project_kernel<T, ZC>), grid, block, 0, s, (const T *)vol, (T *)sino, p->n, p->nz,
                           p->n_angles, p->n_bins, p->d_trig, h, inv_ds, (T)p->atten, accumulate);
    }
    SIPO_LAUNCHED("project_kernel");
    return SIPO_OK;
}

int launch_backproject(sipo_plan p, const void *sino, void *vol, int accumulate, hipStream_t s) {
    return p->dtype == SIPO_F64 ? bp_dispatch<double>(p, sino, vol, accumulate, s)
                                : bp_dispatch<float>(p, sino, vol, accumulate, s);
}

int launch_project(sipo_plan p, const void *vol, void *sino, int accumulate, hipStream_t s) {
    return p->dtype == SIPO_F64 ? fp_dispatch<double>(p, vol, sino, accumulate, s)
                                : fp_dispatch<float>(p, vol, sino, accumulate, s);
}

}  // namespace sipo
