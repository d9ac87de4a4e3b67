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

// P^T over TX x TY voxel tiles.  STAGED: per batch of VB walked views the sinogram window each
// view (and its partner) can send into the tile is copied to LDS first, so the per-voxel gathers
// hit LDS; used when the tile's bin window fits the staged row width.
__host__ __device__ constexpr int bp2d_row_width(int tx, int ty) { return tx + ty <= 40 ? 48 : 80; }

template <typename T, bool STAGED, int TX, int TY, int VB>
__global__ void __launch_bounds__(256) bp2d_kernel(const Geo2D *__restrict__ geo, const int4 *__restrict__ items,
                                                   const T *__restrict__ sino, T *__restrict__ vol, int accumulate) {
    static_assert(TX * TY == 256, "one voxel per thread");
    constexpr int W = bp2d_row_width(TX, TY);
    __shared__ T rows[STAGED ? 2 * VB : 1][STAGED ? W : 1];
    __shared__ int rbase[2 * VB];
    __shared__ double2 vtrig[VB];   // (sin, cos) of the batch's walked views
    // FP32 staged path: per walked view, u at the tile's first voxel relative to each row's first
    // staged bin (the view's, and the mirrored partner's) and u's steps per column and row, split as
    // in taps_rel32, and (sin, cos)
    constexpr bool G32 = STAGED && sizeof(T) == 4;
    __shared__ float vgeo[G32 ? VB : 1][10];
    const int4 it = items[blockIdx.x];
    const Geo2D &g = geo[it.x];
    const int n = g.n, nb = g.n_bins;
    const int c = it.y + (int)(threadIdx.x % TX), r = it.z + (int)(threadIdx.x / TX);
    const bool in_grid = c < n && r < n;
    const bool inside = in_grid && in_vial(c, r, n);
    const double x = centre(c, g.h), y = centre(r, g.h);
    const float xf = (float)x, yf = (float)y;
    const float dcf = (float)(threadIdx.x % TX), drf = (float)(threadIdx.x / TX);
    const T atten = (T)g.atten;
    const T *s0 = sino + g.soff;
    T acc = (T)0;
    for (int k0 = 0; k0 < g.n_walk; k0 += (STAGED ? VB : g.n_walk)) {
        const int nk = STAGED ? min(VB, g.n_walk - k0) : g.n_walk;
        if (STAGED) {
            if ((int)threadIdx.x < 2 * nk) {
                // first staged bin of row (view, mirror): floor of the smallest u over the tile corners, minus 1
                const int kk = k0 + (int)threadIdx.x / 2, mir = threadIdx.x & 1;
                const double2 tr = g.trig[g.walk[kk]];
                const int cx[2] = {it.y, min(it.y + TX, n) - 1}, ry[2] = {it.z, min(it.z + TY, n) - 1};
                double umin = 1e300, umax = -1e300;
                for (int i = 0; i < 2; ++i)
                    for (int j = 0; j < 2; ++j) {
                        const double xs = centre(cx[i], g.h), ys = centre(ry[j], g.h);
                        const double u = fma(fma(-xs, tr.x, ys * tr.y) + 1.0, g.inv_ds, -0.5);
                        umin = fmin(umin, u);
                        umax = fmax(umax, u);
                    }
                const double lo = mir ? (double)(nb - 1) - umax : umin;
                const int rb = (int)floor(lo) - 1;
                rbase[threadIdx.x] = rb;
                if (!mir) vtrig[threadIdx.x / 2] = tr;
                if constexpr (G32) {
                    // once per (tile, view) in FP64; the mirrored row runs along u' = nb - 1 - u
                    const double u00 = fma(fma(-centre(it.y, g.h), tr.x, centre(it.z, g.h) * tr.y) + 1.0, g.inv_ds,
                                           -0.5);
                    float *vg = vgeo[threadIdx.x / 2];
                    const Split32 o = split32(mir ? (double)(nb - 1) - u00 - (double)rb : u00 - (double)rb, kTapScale,
                                              kTapInvScale);
                    vg[mir ? 2 : 0] = o.hi;
                    vg[mir ? 3 : 1] = o.lo;
                    if (!mir) {
                        const Split32 ux = split32(-tr.x * g.h * g.inv_ds, kTapScale, kTapInvScale);
                        const Split32 uy = split32(tr.y * g.h * g.inv_ds, kTapScale, kTapInvScale);
                        vg[4] = ux.hi; vg[5] = ux.lo; vg[6] = uy.hi; vg[7] = uy.lo;
                        vg[8] = (float)tr.x; vg[9] = (float)tr.y;
                    }
                }
            }
            __syncthreads();
            for (int e = threadIdx.x; e < 2 * nk * W; e += 256) {
                const int row = e / W, col = e - row * W;
                const int a = g.walk[k0 + row / 2];
                const int av = (row & 1) ? (g.pair ? g.partner[a] : -1) : a;
                const int b = rbase[row] + col;
                rows[row][col] = (av >= 0 && b >= 0 && b < nb) ? s0[(size_t)av * nb + b] : (T)0;
            }
            __syncthreads();
        }
        if (G32 && inside) {
            // FP32 throughout: the voxel's offsets in the tile against each row's split origin
            for (int kq = 0; kq < nk; ++kq) {
                const float *vg = vgeo[kq];
                const float sn = vg[8], cs = vg[9];
                const float sv = fmaf(-xf, sn, yf * cs), tv = fmaf(xf, cs, yf * sn);
                const Split32 ux{vg[4], vg[5]}, uy{vg[6], vg[7]};
                float w0, w1;
                int bl = taps_rel32(dcf, drf, Split32{vg[0], vg[1]}, ux, uy, sv, tv, (float)atten, w0, w1);
                bl = min(max(bl, 0), W - 2);
                acc = fma((T)w0, rows[2 * kq][bl], acc);
                acc = fma((T)w1, rows[2 * kq][bl + 1], acc);
                if (g.pair) {
                    // opposite view: u' = nb - 1 - u (steps negated), t' = -t, same sqrt(1 - s^2)
                    const Split32 nx{-ux.hi, -ux.lo}, ny{-uy.hi, -uy.lo};
                    bl = taps_rel32(dcf, drf, Split32{vg[2], vg[3]}, nx, ny, sv, -tv, (float)atten, w0, w1);
                    bl = min(max(bl, 0), W - 2);
                    acc = fma((T)w0, rows[2 * kq + 1][bl], acc);
                    acc = fma((T)w1, rows[2 * kq + 1][bl + 1], acc);
                }
            }
        } else if (inside) {
            for (int kq = 0; kq < nk; ++kq) {
                const int a = STAGED ? 0 : g.walk[k0 + kq];
                const double2 tr = STAGED ? vtrig[kq] : g.trig[a];
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
                    T v0, v1;
                    if (STAGED) {
                        const int bl = min(max(b - rbase[2 * kq], 0), W - 2);
                        v0 = rows[2 * kq][bl];
                        v1 = rows[2 * kq][bl + 1];
                    } else {
                        const T *row = s0 + (size_t)a * nb;
                        v0 = (b >= 0 && b < nb) ? row[b] : (T)0;
                        v1 = (b + 1 >= 0 && b + 1 < nb) ? row[b + 1] : (T)0;
                    }
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
                    T v0, v1;
                    if (STAGED) {
                        const int bl = min(max(b - rbase[2 * kq + 1], 0), W - 2);
                        v0 = rows[2 * kq + 1][bl];
                        v1 = rows[2 * kq + 1][bl + 1];
                    } else {
                        const T *row = s0 + (size_t)g.partner[a] * nb;
                        v0 = (b >= 0 && b < nb) ? row[b] : (T)0;
                        v1 = (b + 1 >= 0 && b + 1 < nb) ? row[b + 1] : (T)0;
                    }
                    const T w1 = w * f;
                    acc = fma(w - w1, v0, acc);
                    acc = fma(w1, v1, acc);
                }
            }
        }
        if (STAGED) __syncthreads();
    }
    if (!in_grid) return;
    T *dst = vol + g.voff + (size_t)r * n + c;
    *dst = accumulate ? *dst + acc : acc;
}

template <typename T, int NC, int FB>
__global__ void __launch_bounds__(256) fp2d_kernel(const Geo2D *__restrict__ geo, const int4 *__restrict__ items,
                                                   const T *__restrict__ vol, const T *__restrict__ vol_xt,
                                                   T *__restrict__ sino, int accumulate) {
    extern __shared__ int2 vials[];   // vial extent of every grid line of the instance (n entries)
    const int4 it = items[blockIdx.x];
    const Geo2D &g = geo[it.x];
    const int n = g.n, nb = g.n_bins;
    for (int m = threadIdx.x; m < n; m += 256) vials[m] = g.vial[m];
    __syncthreads();
    const int b = it.z + (int)(threadIdx.x % FB), k = it.y + (int)(threadIdx.x / FB);
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
    const MarchF32 mc32 = march_f32(U00 - (double)b, dU, du, inv_du, s00, dsm, t00, dtm, nb);
    const bool pair = g.pair != 0;
    // along the cross index j the voxels of step m are contiguous in vol ([y][x], y-major rays)
    // or in vol_xt ([x][y], x-major rays); without vol_xt x-major rays read vol with stride n
    const T *base = (xmajor && vol_xt) ? vol_xt + g.voff : vol + g.voff;
    const int sm = xmajor ? (vol_xt ? n : 1) : n, sj = xmajor ? (vol_xt ? 1 : n) : 1;
    T acc1 = (T)0, acc2 = (T)0;
    for (int m = 0; m < n; ++m) {
        const int2 vr = vials[m];
        int jlo;
        T d0, s0, t0;
        if constexpr (sizeof(T) == 4) {
            jlo = march_step_f32(mc32, m, dsj_t, dtj_t, d0, s0, t0);   // FP32 (see MarchF32)
        } else {
            const double U = fma((double)m, dU, U00);
            const double jA = ((double)b - 1.0 - U) * inv_du, jB = ((double)b + 1.0 - U) * inv_du;
            jlo = (int)ceil(fmin(jA, jB) - 1e-9);
            const double jl = (double)jlo;
            d0 = (T)(fma(jl, du, U) - (double)b);
            s0 = (T)fma(jl, dsj, fma((double)m, dsm, s00));
            t0 = (T)fma(jl, dtj, fma((double)m, dtm, t00));
        }
        const T *row = base + m * sm;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const int j = jlo + q;
            const T hat = (T)1 - fabs(d0 + (T)q * du_t);
            if (j < vr.x || j > vr.y || !(hat > (T)0)) continue;
            const T sq = s0 + (T)q * dsj_t;
            T rr = (T)1 - sq * sq;
            rr = rr > (T)0 ? sqrt_t<T>(rr) : (T)0;
            const T tq = t0 + (T)q * dtj_t;
            const T v = row[j * sj];
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

// out[x][y] = in[y][x] per instance, 64 x 64 tiles through LDS.
template <typename T>
__global__ void __launch_bounds__(256) tr2d_kernel(const Geo2D *__restrict__ geo, const int4 *__restrict__ items,
                                                   const T *__restrict__ in, T *__restrict__ out) {
    __shared__ T tile[64][65];
    const int4 it = items[blockIdx.x];
    const Geo2D &g = geo[it.x];
    const int n = g.n;
    const T *src = in + g.voff;
    T *dst = out + g.voff;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {
        const int r = it.z + i, c = it.y + tx;
        tile[i][tx] = (r < n && c < n) ? src[(size_t)r * n + c] : (T)0;
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const int c = it.y + i, r = it.z + tx;
        if (r < n && c < n) dst[(size_t)c * n + r] = tile[tx][i];
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
    g.vial = p->d_vial_rows;
    return g;
}

bool tiles2d_valid(const Tiles2D &t) {
    const bool tile = (t.bx == 32 && t.by == 8) || (t.bx == 16 && t.by == 16) || (t.bx == 64 && t.by == 4);
    return tile && (t.vb == 8 || t.vb == 16 || t.vb == 32) && (t.fb == 32 || t.fb == 64 || t.fb == 128);
}

void append_items_bp2d(const Geo2D &g, int gi, std::vector<int4> &items, const Tiles2D &t) {
    for (int y0 = 0; y0 < g.n; y0 += t.by)
        for (int x0 = 0; x0 < g.n; x0 += t.bx) items.push_back(make_int4(gi, x0, y0, 0));
}

void append_items_tr2d(const Geo2D &g, int gi, std::vector<int4> &items) {
    for (int y0 = 0; y0 < g.n; y0 += 64)
        for (int x0 = 0; x0 < g.n; x0 += 64) items.push_back(make_int4(gi, x0, y0, 0));
}

int launch_tr2d(sipo_dtype dt, const Geo2D *geo, const int4 *items, int n_items, const void *in, void *out,
                hipStream_t s) {
    if (n_items <= 0) return SIPO_OK;
    if (dt == SIPO_F64)
        hipLaunchKernelGGL((tr2d_kernel<double>), dim3(n_items), dim3(256), 0, s, geo, items, (const double *)in,
                           (double *)out);
    else
        hipLaunchKernelGGL((tr2d_kernel<float>), dim3(n_items), dim3(256), 0, s, geo, items, (const float *)in,
                           (float *)out);
    SIPO_LAUNCHED("tr2d_kernel");
    return SIPO_OK;
}

void append_items_fp2d(const Geo2D &g, int gi, std::vector<int4> &items, const Tiles2D &t) {
    for (int k0 = 0; k0 < g.n_walk; k0 += t.fv())
        for (int b0 = 0; b0 < g.n_bins; b0 += t.fb) items.push_back(make_int4(gi, k0, b0, 0));
}

// The tile's bin window (with guards) fits the staged row width for this detector/grid ratio.
bool bp2d_stage_fits(int n, int n_bins, const Tiles2D &t) {
    const double span = std::sqrt((double)(t.bx - 1) * (t.bx - 1) + (double)(t.by - 1) * (t.by - 1)) * n_bins / n;
    return span + 5.0 <= (double)bp2d_row_width(t.bx, t.by);
}

template <typename T, bool STAGED, int TX, int TY>
static void bp2d_vb(const Tiles2D &t, dim3 grid, const Geo2D *geo, const int4 *items, const void *sino, void *vol,
                    int accumulate, hipStream_t s) {
    switch (t.vb) {
        case 8: hipLaunchKernelGGL((bp2d_kernel<T, STAGED, TX, TY, 8>), grid, dim3(256), 0, s, geo, items,
                                   (const T *)sino, (T *)vol, accumulate); break;
        case 32: hipLaunchKernelGGL((bp2d_kernel<T, STAGED, TX, TY, 32>), grid, dim3(256), 0, s, geo, items,
                                    (const T *)sino, (T *)vol, accumulate); break;
        default: hipLaunchKernelGGL((bp2d_kernel<T, STAGED, TX, TY, 16>), grid, dim3(256), 0, s, geo, items,
                                    (const T *)sino, (T *)vol, accumulate); break;
    }
}

int launch_bp2d(sipo_dtype dt, bool staged, const Geo2D *geo, const int4 *items, int n_items, const void *sino,
                void *vol, int accumulate, hipStream_t s, const Tiles2D &t) {
    if (n_items <= 0) return SIPO_OK;
    if (!tiles2d_valid(t)) return fail(SIPO_E_INVALID, "2D backprojector: unsupported tile %d x %d, %d views", t.bx,
                                       t.by, t.vb);
    const dim3 grid(n_items);
    if (dt == SIPO_F64 || !staged) {
        // the other shapes serve FP32 staged launches only
        if (!t.is_default())
            return fail(SIPO_E_UNSUPPORTED, "2D backprojector: %d x %d tiles need an FP32 staged launch", t.bx, t.by);
        if (dt == SIPO_F64) {
            if (staged) bp2d_vb<double, true, 32, 8>(t, grid, geo, items, sino, vol, accumulate, s);
            else bp2d_vb<double, false, 32, 8>(t, grid, geo, items, sino, vol, accumulate, s);
        } else {
            bp2d_vb<float, false, 32, 8>(t, grid, geo, items, sino, vol, accumulate, s);
        }
    } else if (t.bx == 16) {
        bp2d_vb<float, true, 16, 16>(t, grid, geo, items, sino, vol, accumulate, s);
    } else if (t.bx == 64) {
        bp2d_vb<float, true, 64, 4>(t, grid, geo, items, sino, vol, accumulate, s);
    } else {
        bp2d_vb<float, true, 32, 8>(t, grid, geo, items, sino, vol, accumulate, s);
    }
    SIPO_LAUNCHED("bp2d_kernel");
    return SIPO_OK;
}

template <typename T, int FB>
static int fp2d_t(int nc, int n_max, const Geo2D *geo, const int4 *items, int n_items, const void *vol,
                  const void *vol_xt, void *sino, int accumulate, hipStream_t s) {
    const dim3 grid(n_items), block(256);
    const size_t shm = sizeof(int2) * (size_t)n_max;
    const T *v = (const T *)vol, *vx = (const T *)vol_xt;
    switch (nc) {
        case 3: hipLaunchKernelGGL((fp2d_kernel<T, 3, FB>), grid, block, shm, s, geo, items, v, vx, (T *)sino,
                                   accumulate); break;
        case 4: hipLaunchKernelGGL((fp2d_kernel<T, 4, FB>), grid, block, shm, s, geo, items, v, vx, (T *)sino,
                                   accumulate); break;
        case 6: hipLaunchKernelGGL((fp2d_kernel<T, 6, FB>), grid, block, shm, s, geo, items, v, vx, (T *)sino,
                                   accumulate); break;
        default: return fail(SIPO_E_UNSUPPORTED, "2D projector: unsupported candidate count %d", nc);
    }
    SIPO_LAUNCHED("fp2d_kernel");
    return SIPO_OK;
}

int launch_fp2d(sipo_dtype dt, int nc, int n_max, const Geo2D *geo, const int4 *items, int n_items, const void *vol,
                const void *vol_xt, void *sino, int accumulate, hipStream_t s, const Tiles2D &t) {
    if (n_items <= 0) return SIPO_OK;
    if (n_max < 1 || n_max > kF2MaxN) return fail(SIPO_E_UNSUPPORTED, "2D projector: grid %d > %d", n_max, kF2MaxN);
    if (!tiles2d_valid(t)) return fail(SIPO_E_INVALID, "2D projector: unsupported bundle of %d bins", t.fb);
    if (dt == SIPO_F64) {
        if (t.fb != 64) return fail(SIPO_E_UNSUPPORTED, "2D projector: %d-bin bundles need FP32", t.fb);
        return fp2d_t<double, 64>(nc, n_max, geo, items, n_items, vol, vol_xt, sino, accumulate, s);
    }
    switch (t.fb) {
        case 32: return fp2d_t<float, 32>(nc, n_max, geo, items, n_items, vol, vol_xt, sino, accumulate, s);
        case 128: return fp2d_t<float, 128>(nc, n_max, geo, items, n_items, vol, vol_xt, sino, accumulate, s);
        default: return fp2d_t<float, 64>(nc, n_max, geo, items, n_items, vol, vol_xt, sino, accumulate, s);
    }
}

// The plan as a one-instance batch (single-slice plans only).
int plan_build_2d(sipo_plan p) {
    p->p2d_ok = p->nz == 1 && p->p3d_nc > 0 && p->n <= kF2MaxN;
    if (!p->p2d_ok) return SIPO_OK;
    const Geo2D g = plan_geo2d(p, 0, 0);
    std::vector<int4> ib, ifp, itr;
    append_items_bp2d(g, 0, ib);
    append_items_fp2d(g, 0, ifp);
    append_items_tr2d(g, 0, itr);
    SIPO_TRY(plan_alloc(p, (void **)&p->d_geo2d, sizeof(Geo2D)));
    SIPO_TRY(plan_alloc(p, (void **)&p->d_items_bp2d, sizeof(int4) * ib.size()));
    SIPO_TRY(plan_alloc(p, (void **)&p->d_items_fp2d, sizeof(int4) * ifp.size()));
    SIPO_HIP(hipMemcpy(p->d_geo2d, &g, sizeof(Geo2D), hipMemcpyHostToDevice));
    SIPO_HIP(hipMemcpy(p->d_items_bp2d, ib.data(), sizeof(int4) * ib.size(), hipMemcpyHostToDevice));
    SIPO_HIP(hipMemcpy(p->d_items_fp2d, ifp.data(), sizeof(int4) * ifp.size(), hipMemcpyHostToDevice));
    SIPO_TRY(plan_alloc(p, (void **)&p->d_items_tr2d, sizeof(int4) * itr.size()));
    SIPO_HIP(hipMemcpy(p->d_items_tr2d, itr.data(), sizeof(int4) * itr.size(), hipMemcpyHostToDevice));
    p->n_items_bp2d = (int)ib.size();
    p->n_items_fp2d = (int)ifp.size();
    p->n_items_tr2d = (int)itr.size();
    return SIPO_OK;
}

}  // namespace sipo
