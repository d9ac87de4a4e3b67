// Single-slice (2D) projector pair P^T / P (Eq. 2-3), batched over instances.
//
// A launch covers any number of instances of different grid size, view count
// and detector width: each workgroup takes one work item naming its instance
// (a Geo2D record) and its tile.  This is how many small problems fill the
// chip in one launch; a single plan is the one-instance case.
//
//   P^T: a workgroup owns a 32 x 8 voxel tile; per walked view a thread
//        evaluates its voxel's interpolation taps once and gathers two bins
//        (and, for an opposite pair, the two mirrored bins of the partner view
//        with the same s, u and sqrt(1 - s^2), only the depth t changing sign).
//   P:   a workgroup owns 64 bins x 4 walked views; a thread walks its ray
//        along the grid axis the ray is most aligned with and, per step, takes
//        the NC voxels whose hat weight max(0, 1 - |u - b|) can be positive
//        (the partner ray, bin nb - 1 - b, sees the same voxels and weights).
//
// No atomics: every output element is written by one thread, so results are
// reproducible run to run.
#include <algorithm>
#include <vector>

#include "sipo_internal.hpp"

namespace sipo {

__device__ __forceinline__ bool in_vial(int c, int r, int n) {
    const long long a = 2LL * c + 1 - n, b = 2LL * r + 1 - n;
    return a * a + b * b <= (long long)n * n;
}

template <typename T>
__global__ void __launch_bounds__(256) bp2d_kernel(const Geo2D *__restrict__ geo, const int4 *__restrict__ items,
                                                   const T *__restrict__ sino, T *__restrict__ vol, int accumulate) {
    const int4 it = items[blockIdx.x];
    const Geo2D &g = geo[it.x];
    const int n = g.n, nb = g.n_bins;
    const int c = it.y + (int)(threadIdx.x % kB2X), r = it.z + (int)(threadIdx.x / kB2X);
    if (c >= n || r >= n) return;
    T acc = (T)0;
    if (in_vial(c, r, n)) {
        const double x = centre(c, g.h), y = centre(r, g.h);
        const T atten = (T)g.atten;
        const T *s0 = sino + g.soff;
        for (int k = 0; k < g.n_walk; ++k) {
            const int a = g.walk[k];
            const double2 tr = g.trig[a];
            const double s = fma(-x, tr.x, y * tr.y);
            const double u = fma(s + 1.0, g.inv_ds, -0.5);
            const double t = fma(x, tr.y, y * tr.x);
            T rr = (T)fma(-s, s, 1.0);
            rr = rr > (T)0 ? sqrt_t<T>(rr) : (T)0;
            {
                const double bf = floor(u);
                const int b = (int)bf;
                const T f = (T)(u - bf);
                const T w = exp_neg<T>(atten, (T)t + rr);
                const T *row = s0 + (size_t)a * nb;
                const T v0 = (b >= 0 && b < nb) ? row[b] : (T)0;
                const T v1 = (b + 1 >= 0 && b + 1 < nb) ? row[b + 1] : (T)0;
                const T w1 = w * f;
                acc = fma(w - w1, v0, acc);
                acc = fma(w1, v1, acc);
            }
            if (g.pair) {
                // opposite view: u' = nb - 1 - u, t' = -t, same sqrt(1 - s^2)
                const double u2 = (double)(nb - 1) - u;
                const double bf = floor(u2);
                const int b = (int)bf;
                const T f = (T)(u2 - bf);
                const T w = exp_neg<T>(atten, rr - (T)t);
                const T *row = s0 + (size_t)g.partner[a] * nb;
                const T v0 = (b >= 0 && b < nb) ? row[b] : (T)0;
                const T v1 = (b + 1 >= 0 && b + 1 < nb) ? row[b + 1] : (T)0;
                const T w1 = w * f;
                acc = fma(w - w1, v0, acc);
                acc = fma(w1, v1, acc);
            }
        }
    }
    T *dst = vol + g.voff + (size_t)r * n + c;
    *dst = accumulate ? *dst + acc : acc;
}

template <typename T, int NC>
__global__ void __launch_bounds__(256) fp2d_kernel(const Geo2D *__restrict__ geo, const int4 *__restrict__ items,
                                                   const T *__restrict__ vol, T *__restrict__ sino, int accumulate) {
    const int4 it = items[blockIdx.x];
    const Geo2D &g = geo[it.x];
    const int n = g.n, nb = g.n_bins;
    const int b = it.z + (int)(threadIdx.x % kF2B), k = it.y + (int)(threadIdx.x / kF2B);
    if (b >= nb || k >= g.n_walk) return;
    const int a = g.walk[k];
    const double2 tr = g.trig[a];
    const double sn = tr.x, cs = tr.y;
    const bool xmajor = fabs(cs) >= fabs(sn);
    // affine frame: s(m, j) = s00 + m dsm + j dsj, t likewise, u = (s + 1) inv_ds - 1/2
    const double h = g.h, inv_ds = g.inv_ds;
    const double c0 = centre(0, h);
    const double s00 = fma(-c0, sn, c0 * cs), t00 = fma(c0, cs, c0 * sn);
    const double dsj = (xmajor ? cs : -sn) * h, dsm = (xmajor ? -sn : cs) * h;
    const double dtj = (xmajor ? sn : cs) * h, dtm = (xmajor ? cs : sn) * h;
    const double du = dsj * inv_ds, dU = dsm * inv_ds, U00 = fma(s00 + 1.0, inv_ds, -0.5);
    const double inv_du = 1.0 / du;
    const T du_t = (T)du, dsj_t = (T)dsj, dtj_t = (T)dtj, atten = (T)g.atten;
    const bool pair = g.pair != 0;
    const T *v0 = vol + g.voff;
    T acc1 = (T)0, acc2 = (T)0;
    for (int m = 0; m < n; ++m) {
        const double U = fma((double)m, dU, U00);
        const double jA = ((double)b - 1.0 - U) * inv_du, jB = ((double)b + 1.0 - U) * inv_du;
        const int jlo = (int)ceil(fmin(jA, jB) - 1e-9);
        const double jl = (double)jlo;
        const T d0 = (T)(fma(jl, du, U) - (double)b);
        const T s0 = (T)fma(jl, dsj, fma((double)m, dsm, s00));
        const T t0 = (T)fma(jl, dtj, fma((double)m, dtm, t00));
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const int j = jlo + q;
            const int c = xmajor ? m : j, r = xmajor ? j : m;
            const T hat = (T)1 - fabs(d0 + (T)q * du_t);
            if (j < 0 || j >= n || !(hat > (T)0) || !in_vial(c, r, n)) continue;
            const T sq = s0 + (T)q * dsj_t;
            T rr = (T)1 - sq * sq;
            rr = rr > (T)0 ? sqrt_t<T>(rr) : (T)0;
            const T tq = t0 + (T)q * dtj_t;
            const T v = v0[(size_t)r * n + c];
            acc1 = fma(hat * exp_neg<T>(atten, tq + rr), v, acc1);
            if (pair) acc2 = fma(hat * exp_neg<T>(atten, rr - tq), v, acc2);
        }
    }
    T *d1 = sino + g.soff + (size_t)a * nb + b;
    *d1 = accumulate ? *d1 + acc1 : acc1;
    if (pair) {
        T *d2 = sino + g.soff + (size_t)g.partner[a] * nb + (nb - 1 - b);
        *d2 = accumulate ? *d2 + acc2 : acc2;
    }
}

// ------------------------------------------------------------------ host side
Geo2D plan_geo2d(sipo_plan p, long long soff, long long voff) {
    Geo2D g{};
    g.trig = p->d_trig;
    g.walk = p->d_angle_order;
    g.partner = p->d_partner;
    g.soff = soff;
    g.voff = voff;
    g.n = p->n;
    g.n_angles = p->n_angles;
    g.n_bins = p->n_bins;
    g.n_walk = p->n_walk;
    g.pair = p->p3d_pair ? 1 : 0;
    g.nc = p->p3d_nc;
    g.h = 2.0 / p->n;
    g.inv_ds = 0.5 * p->n_bins;
    g.atten = p->atten;
    return g;
}

void append_items_bp2d(const Geo2D &g, int gi, std::vector<int4> &items) {
    for (int y0 = 0; y0 < g.n; y0 += kB2Y)
        for (int x0 = 0; x0 < g.n; x0 += kB2X) items.push_back(make_int4(gi, x0, y0, 0));
}

void append_items_fp2d(const Geo2D &g, int gi, std::vector<int4> &items) {
    for (int k0 = 0; k0 < g.n_walk; k0 += kF2V)
        for (int b0 = 0; b0 < g.n_bins; b0 += kF2B) items.push_back(make_int4(gi, k0, b0, 0));
}

int launch_bp2d(sipo_dtype dt, const Geo2D *geo, const int4 *items, int n_items, const void *sino, void *vol,
                int accumulate, hipStream_t s) {
    if (n_items <= 0) return SIPO_OK;
    if (dt == SIPO_F64)
        hipLaunchKernelGGL((bp2d_kernel<double>), dim3(n_items), dim3(256), 0, s, geo, items, (const double *)sino,
                           (double *)vol, accumulate);
    else
        hipLaunchKernelGGL((bp2d_kernel<float>), dim3(n_items), dim3(256), 0, s, geo, items, (const float *)sino,
                           (float *)vol, accumulate);
    SIPO_LAUNCHED("bp2d_kernel");
    return SIPO_OK;
}

template <typename T>
static int fp2d_t(int nc, const Geo2D *geo, const int4 *items, int n_items, const void *vol, void *sino,
                  int accumulate, hipStream_t s) {
    const dim3 grid(n_items), block(256);
    switch (nc) {
        case 3: hipLaunchKernelGGL((fp2d_kernel<T, 3>), grid, block, 0, s, geo, items, (const T *)vol, (T *)sino,
                                   accumulate); break;
        case 4: hipLaunchKernelGGL((fp2d_kernel<T, 4>), grid, block, 0, s, geo, items, (const T *)vol, (T *)sino,
                                   accumulate); break;
        case 6: hipLaunchKernelGGL((fp2d_kernel<T, 6>), grid, block, 0, s, geo, items, (const T *)vol, (T *)sino,
                                   accumulate); break;
        default: return fail(SIPO_E_UNSUPPORTED, "2D projector: unsupported candidate count %d", nc);
    }
    SIPO_LAUNCHED("fp2d_kernel");
    return SIPO_OK;
}

int launch_fp2d(sipo_dtype dt, int nc, const Geo2D *geo, const int4 *items, int n_items, const void *vol,
                void *sino, int accumulate, hipStream_t s) {
    if (n_items <= 0) return SIPO_OK;
    return dt == SIPO_F64 ? fp2d_t<double>(nc, geo, items, n_items, vol, sino, accumulate, s)
                          : fp2d_t<float>(nc, geo, items, n_items, vol, sino, accumulate, s);
}

// The plan as a one-instance batch (single-slice plans only).
int plan_build_2d(sipo_plan p) {
    p->p2d_ok = p->nz == 1 && p->p3d_nc > 0;
    if (!p->p2d_ok) return SIPO_OK;
    const Geo2D g = plan_geo2d(p, 0, 0);
    std::vector<int4> ib, ifp;
    append_items_bp2d(g, 0, ib);
    append_items_fp2d(g, 0, ifp);
    SIPO_HIP(hipMalloc(&p->d_geo2d, sizeof(Geo2D)));
    SIPO_HIP(hipMalloc(&p->d_items_bp2d, sizeof(int4) * ib.size()));
    SIPO_HIP(hipMalloc(&p->d_items_fp2d, sizeof(int4) * ifp.size()));
    SIPO_HIP(hipMemcpy(p->d_geo2d, &g, sizeof(Geo2D), hipMemcpyHostToDevice));
    SIPO_HIP(hipMemcpy(p->d_items_bp2d, ib.data(), sizeof(int4) * ib.size(), hipMemcpyHostToDevice));
    SIPO_HIP(hipMemcpy(p->d_items_fp2d, ifp.data(), sizeof(int4) * ifp.size(), hipMemcpyHostToDevice));
    p->n_items_bp2d = (int)ib.size();
    p->n_items_fp2d = (int)ifp.size();
    return SIPO_OK;
}

}  // namespace sipo
