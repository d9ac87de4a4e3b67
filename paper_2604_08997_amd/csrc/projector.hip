// Backprojector P^T and projector P (Eq. 2-3): gathers in both directions.
//
// Slice kernels (nz == 1, and the general fallback):
//   P^T: one thread per voxel (x, y) and a chunk of ZC slices; per view the two
//        interpolation taps are computed once and the two sinogram samples
//        of every slice in the chunk are gathered.
//   P:   one thread per (bin, view) and a chunk of ZC slices; the ray is
//        walked along its major axis and, per step, the few voxels whose taps
//        can reach the bin are tested with the same tap function as P^T.
//
// Volume kernels (nz > 1): LDS-staged, z-contiguous layouts (see below).
#include <algorithm>
#include <vector>

#include "sipo_internal.hpp"

namespace sipo {

template <typename T>
struct Vec4;
template <>
struct Vec4<float> { using type = float4; };
template <>
struct Vec4<double> { using type = double4; };

// Exact integer form of "voxel centre inside the closed unit disk":
// ((2c+1-n)^2 + (2r+1-n)^2 <= n^2) <=> x^2 + y^2 <= 1 with x = -1 + (c+1/2) 2/n.
__device__ __forceinline__ bool vial_ij(int c, int r, int n) {
    const long long a = 2LL * c + 1 - n, b = 2LL * r + 1 - n;
    return a * a + b * b <= (long long)n * n;
}

// ------------------------------------------------------------- slice kernels
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
    if (vial_ij(c, r, n)) {
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
        const double pm = centre(i, h);
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
            if (!vial_ij(c, r, n)) continue;
            const double x = centre(c, h), y = centre(r, h);
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

// ------------------------------------------------------------------ 3D P^T
// Input sinogram [view][bin][z].  One workgroup = a 32 x 16 voxel tile and ZC
// slices; 256 threads, each owning two voxels (rows ty, ty + 8) and ZC slices
// in registers.  Views go in batches of kBpTB: for each view the bins the tile
// can reach (floor(u_min) - 1 .. floor(u_max) + 2 over the tile, at most kBpW)
// are copied into LDS as [view][bin][z] rows -- a straight copy of
// z-contiguous 16-byte chunks -- padded by 4 elements so that the rows read
// by the 16 lanes of one LDS pass land in different banks.  A voxel then reads
// four slices of each tap bin per 128-bit load.  Bins outside the detector are
// staged as zeros, so the inner loop has no bounds tests.
// runs of y tiles kept together: view batches for the projector, rows for the backprojector
constexpr int kXcdRunP = 1, kXcdRunBp = 0;

constexpr int kBpTX = 32, kBpTY = 16, kBpTB = 6, kBpW = 40;

static bool bp3d_fits(int n, int nb) {
    const double span = std::sqrt((double)(kBpTX - 1) * (kBpTX - 1) + (double)(kBpTY - 1) * (kBpTY - 1)) * nb / n;
    return span + 5.0 <= (double)kBpW;
}

// VEC (nz a multiple of 4, at most 16 slices per thread): the staging of a view batch issues every
// b128 load of the window at once, from addresses clamped into the sinogram, and zeroes the values
// outside it as they are written to LDS, so the loads carry no branches and a thread waits once per
// batch.  Otherwise the window is staged word by word with guarded loads (at 32 slices per thread
// the registers of a whole window would cost a wave per SIMD).  Either way the next batch's
// (sin, cos) is fetched during the current batch.
template <typename T, int ZC, bool VEC>
__global__ void __launch_bounds__(256) backproject3d_kernel(const T *__restrict__ sino_t, T *__restrict__ vol, int n,
                                                            int nz, int n_angles, int nb,
                                                            const double2 *__restrict__ trig, double h,
                                                            double inv_ds, T atten, int accumulate,
                                                            const uint8_t *__restrict__ tile_on, int nsplit,
                                                            long long split_stride,
                                                            const uint8_t *__restrict__ need) {
    using V4 = typename Vec4<T>::type;
    constexpr int Z4 = ZC / 4, ZP = ZC + 4;
    __shared__ __align__(16) T lds[kBpTB][kBpW][ZP];
    __shared__ int bmin_s[kBpTB];
    // FP32: per view of the batch, the detector coordinate at the tile's origin relative to its first
    // staged bin and its increments per column and row (hi / lo splits, see taps_rel32), and (sin, cos)
    __shared__ float geo_s[sizeof(T) == 4 ? kBpTB : 1][8];
    // a wave owns two 8 x 8 blocks of the tile's 32 x 16 columns (rows ty and ty + 8 of its 8 columns):
    // compact blocks let whole waves skip where the needed voxels end (need)
    const int tx = ((threadIdx.x >> 6) << 3) | (threadIdx.x & 7), ty = (threadIdx.x >> 3) & 7;
    // grid.z = z chunks x view splits; split s sums its share of the views into partial sum s
    const int3 tile = xcd_tile<kXcdRunBp>();
    const int nzc = gridDim.z / nsplit, zb = tile.z % nzc, split = tile.z / nzc;
    const int x0 = tile.x * kBpTX, y0 = tile.y * kBpTY, z0 = zb * ZC;
    const int c = x0 + tx;
    const int r[2] = {y0 + ty, y0 + ty + 8};
    if (tile_on && !tile_on[((size_t)zb * gridDim.y + tile.y) * gridDim.x + tile.x]) {
        // no voxel of the tile is needed: write zeros (or leave an accumulated output as it is);
        // with splits the reduction writes those zeros
        if (!accumulate && nsplit == 1)
            for (int j = 0; j < 2; ++j)
                if (c < n && r[j] < n)
                    for (int k = 0; k < ZC && z0 + k < nz; ++k) vol[((size_t)(z0 + k) * n + r[j]) * n + c] = (T)0;
        return;
    }
    const double xv = centre(c, h);
    const double yv[2] = {centre(r[0], h), centre(r[1], h)};
    const float xf = (float)xv, yf[2] = {(float)yv[0], (float)yv[1]};
    const float dcf = (float)tx, drf[2] = {(float)ty, (float)(ty + 8)};
    // need (masked solves): per z chunk and column, whether any of the column's voxels in the chunk
    // is read; the lanes of the others skip the sum and store zero, and a wave whose lanes all skip
    // issues no LDS reads or FMAs
    bool inside[2];
#pragma unroll
    for (int j = 0; j < 2; ++j)
        inside[j] = c < n && r[j] < n && vial_ij(c, r[j], n) && (!need || need[((size_t)zb * n + r[j]) * n + c]);
    T acc[2][ZC];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int k = 0; k < ZC; ++k) acc[j][k] = (T)0;
    const int cx1 = min(x0 + kBpTX, n) - 1, cy1 = min(y0 + kBpTY, n) - 1;
    const int nvb = (n_angles + kBpTB - 1) / kBpTB, per = (nvb + nsplit - 1) / nsplit;
    const int a_beg = split * per * kBpTB, a_end = min(n_angles, (split + 1) * per * kBpTB);
    double2 tr_next = trig[min(a_beg + (int)threadIdx.x, n_angles - 1)];
    for (int a0 = a_beg; a0 < a_end; a0 += kBpTB) {
        const int na = min(kBpTB, a_end - a0);
        if ((int)threadIdx.x < na) {
            const double2 tr = tr_next;
            double umin = 1e300;
            const int cs_[2] = {x0, cx1}, rs_[2] = {y0, cy1};
            for (int i = 0; i < 2; ++i)
                for (int k = 0; k < 2; ++k) {
                    const double s = fma(-centre(cs_[i], h), tr.x, centre(rs_[k], h) * tr.y);
                    umin = fmin(umin, fma(s + 1.0, inv_ds, -0.5));
                }
            const int bm = (int)floor(umin) - 1;
            bmin_s[threadIdx.x] = bm;
            if constexpr (sizeof(T) == 4) {
                // once per (tile, view) in FP64: u at the tile's first voxel relative to bm, and its
                // steps per column and per row
                const double s0 = fma(-centre(x0, h), tr.x, centre(y0, h) * tr.y);
                const Split32 u0 = split32(fma(s0 + 1.0, inv_ds, -0.5) - (double)bm, kTapScale, kTapInvScale);
                const Split32 ux = split32(-tr.x * h * inv_ds, kTapScale, kTapInvScale);
                const Split32 uy = split32(tr.y * h * inv_ds, kTapScale, kTapInvScale);
                float *g = geo_s[threadIdx.x];
                g[0] = u0.hi; g[1] = u0.lo; g[2] = ux.hi; g[3] = ux.lo; g[4] = uy.hi; g[5] = uy.lo;
                g[6] = (float)tr.x; g[7] = (float)tr.y;
            }
        }
        __syncthreads();
        const int tot = na * kBpW * Z4;
        if constexpr (VEC) {
            constexpr int NE = (kBpTB * kBpW * Z4 + 255) / 256;   // b128 words per thread and batch
            V4 wv[NE];
#pragma unroll
            for (int i = 0; i < NE; ++i) {
                const int e = min((int)threadIdx.x + 256 * i, tot - 1);
                const int z4 = e % Z4, rest = e / Z4, b = rest % kBpW, k = rest / kBpW;
                const int gb = min(max(bmin_s[k] + b, 0), nb - 1), gz = min(z0 + 4 * z4, nz - 4);
                wv[i] = *(const V4 *)(sino_t + ((size_t)(a0 + k) * nb + gb) * nz + gz);   // 16-byte aligned
            }
            tr_next = trig[min(a0 + kBpTB + (int)threadIdx.x, n_angles - 1)];
#pragma unroll
            for (int i = 0; i < NE; ++i) {
                const int e = (int)threadIdx.x + 256 * i;
                if (e < tot) {
                    const int z4 = e % Z4, rest = e / Z4, b = rest % kBpW, k = rest / kBpW;
                    const int gb = bmin_s[k] + b, gz = z0 + 4 * z4;
                    const bool ok = gb >= 0 && gb < nb && gz < nz;
                    V4 v = wv[i];
                    T *vv = (T *)&v;
#pragma unroll
                    for (int q = 0; q < 4; ++q) vv[q] = ok ? vv[q] : (T)0;
                    *(V4 *)&lds[k][b][4 * z4] = v;
                }
            }
        } else {
            for (int e = threadIdx.x; e < tot; e += 256) {
                const int z4 = e % Z4;
                const int rest = e / Z4;
                const int b = rest % kBpW;
                const int k = rest / kBpW;
                const int gb = bmin_s[k] + b, gz = z0 + 4 * z4;
                V4 v;
                T *vv = (T *)&v;
                if (gb >= 0 && gb < nb) {
                    const T *src = sino_t + ((size_t)(a0 + k) * nb + gb) * nz + gz;
                    if ((nz & 3) == 0 && gz + 3 < nz) {
                        v = *(const V4 *)src;   // 16-byte aligned: nz % 4 == 0
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q) vv[q] = (gz + q < nz) ? src[q] : (T)0;
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) vv[q] = (T)0;
                }
                *(V4 *)&lds[k][b][4 * z4] = v;
            }
            tr_next = trig[min(a0 + kBpTB + (int)threadIdx.x, n_angles - 1)];
        }
        __syncthreads();
        for (int k = 0; k < na; ++k) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                if (!inside[j]) continue;
                T w0, w1;
                int br;
                if constexpr (sizeof(T) == 4) {
                    // FP32 throughout: the voxel's offsets in the tile against the view's split origin
                    const float *g = geo_s[k];
                    const float sn = g[6], cs = g[7];
                    const float sv = fmaf(-xf, sn, yf[j] * cs), tv = fmaf(xf, cs, yf[j] * sn);
                    br = taps_rel32(dcf, drf[j], Split32{g[0], g[1]}, Split32{g[2], g[3]}, Split32{g[4], g[5]}, sv, tv,
                                    (float)atten, w0, w1);
                } else {
                    const double2 tr = trig[a0 + k];
                    br = taps<T>(xv, yv[j], tr.x, tr.y, inv_ds, atten, w0, w1) - bmin_s[k];
                }
                const T *row0 = &lds[k][br][0];
                const T *row1 = &lds[k][br + 1][0];
#pragma unroll
                for (int z4 = 0; z4 < Z4; ++z4) {
                    const V4 s0 = *(const V4 *)(row0 + 4 * z4);
                    const V4 s1 = *(const V4 *)(row1 + 4 * z4);
                    acc[j][4 * z4 + 0] = fma(w1, s1.x, fma(w0, s0.x, acc[j][4 * z4 + 0]));
                    acc[j][4 * z4 + 1] = fma(w1, s1.y, fma(w0, s0.y, acc[j][4 * z4 + 1]));
                    acc[j][4 * z4 + 2] = fma(w1, s1.z, fma(w0, s0.z, acc[j][4 * z4 + 2]));
                    acc[j][4 * z4 + 3] = fma(w1, s1.w, fma(w0, s0.w, acc[j][4 * z4 + 3]));
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        if (c >= n || r[j] >= n) continue;
#pragma unroll
        for (int k = 0; k < ZC; ++k) {
            if (z0 + k < nz) {
                const size_t idx = (size_t)split * split_stride + ((size_t)(z0 + k) * n + r[j]) * n + c;
                vol[idx] = accumulate ? vol[idx] + acc[j][k] : acc[j][k];
            }
        }
    }
}

// Sum of the view splits' partial volumes on switched-on tiles (fixed order); switched-off tiles get
// zeros, or with keep_off are left as they are.
template <typename T, int ZC>
__global__ void __launch_bounds__(256) k_bp3d_reduce(const T *__restrict__ part, T *__restrict__ vol,
                                                     const uint8_t *__restrict__ tile_on, int n, int nz, int nsplit,
                                                     long long total, int keep_off) {
    // one workgroup per backprojector tile (grid = the backprojector's tiles): a thread owns voxel x of
    // rows y and y + 8 in every slice of the tile.  Per group of up to 8 slices, a split's 2 x 8 values
    // are loaded together, from addresses clamped into the volume (rows or slices past its edge are
    // loaded but never stored), so the loads carry no branches and the thread waits once per split;
    // every sum adds the splits in order 0, 1, ...
    constexpr int G = ZC < 8 ? ZC : 8;
    const int3 tile = xcd_tile<0>();
    const bool on = !tile_on || tile_on[((size_t)tile.z * gridDim.y + tile.y) * gridDim.x + tile.x];
    if (!on && keep_off) return;
    const int x = tile.x * kBpTX + (threadIdx.x & 31), y = tile.y * kBpTY + (threadIdx.x >> 5);
    if (x >= n) return;
    const int ya = min(y, n - 1), yb = min(y + 8, n - 1);
    for (int z0 = tile.z * ZC; z0 < min(nz, (tile.z + 1) * ZC); z0 += G) {
        size_t at[G][2];
#pragma unroll
        for (int k = 0; k < G; ++k) {
            const size_t zz = (size_t)min(z0 + k, nz - 1) * n;
            at[k][0] = (zz + ya) * n + x;
            at[k][1] = (zz + yb) * n + x;
        }
        T v[G][2];
#pragma unroll
        for (int k = 0; k < G; ++k) v[k][0] = v[k][1] = (T)0;
        if (on)
            for (int s = 0; s < nsplit; ++s) {
                const T *ps = part + (size_t)s * total;
                T t[G][2];
#pragma unroll
                for (int k = 0; k < G; ++k)
#pragma unroll
                    for (int h = 0; h < 2; ++h) t[k][h] = ps[at[k][h]];
#pragma unroll
                for (int k = 0; k < G; ++k)
#pragma unroll
                    for (int h = 0; h < 2; ++h) v[k][h] += t[k][h];
            }
#pragma unroll
        for (int k = 0; k < G; ++k)
#pragma unroll
            for (int h = 0; h < 2; ++h)
                if (z0 + k < nz && y + 8 * h < n) vol[at[k][h]] = v[k][h];
    }
}

// ------------------------------------------------------------------- 3D P
// Input volume [y][x][z], output sinogram [view][bin][z].  One workgroup = a
// bundle of kPB = 32 neighbouring bins x up to kPV = 8 views that march along
// the same grid axis (consecutive in the plan's view order) x ZC slices.
// Thread = one (bin, view) ray with ZC accumulators.  The bundle walks the
// march axis kPCM steps at a time; for each chunk the union of the cross-axis
// ranges the bundle can reach is staged in LDS as [step][z/4][cross][4]
// (coalesced copies of z-contiguous chunks; voxels outside the vial are staged
// as zeros, which is where their columns of P vanish).  Along the cross axis
// the detector coordinate s, the depth t and u move linearly, so per step a
// ray takes its NC candidate voxels j = jlo .. jlo + NC - 1 and weights each by
// a_j max(0, 1 - |u_j - b|); a candidate outside the ray's reach gets weight 0
// (no divergence).
//
// PAIR: every view comes with its opposite view (theta + pi).  The opposite
// ray of bin b is bin nb - 1 - b: it meets the same voxels with the same
// interpolation weights (s and t change sign), so one staged operand feeds
// both rays and only the attenuation factor is evaluated twice.
//
// The host splits view batches so the staged range never exceeds kPCR.
template <typename T, int ZC, int NC, bool PAIR>
__global__ void __launch_bounds__(256) project3d_kernel(const T *__restrict__ vol_t, T *__restrict__ sino_t, int n,
                                                        int nz, int nb, const double2 *__restrict__ trig,
                                                        const int *__restrict__ order,
                                                        const int *__restrict__ partner,
                                                        const int4 *__restrict__ batches, double h, double inv_ds,
                                                        T atten, const uint8_t *__restrict__ wg_on) {
    using V4 = typename Vec4<T>::type;
    constexpr int Z4 = ZC / 4;
    constexpr int NR = PAIR ? 2 : 1;
    __shared__ V4 lds[kPCM][Z4][kPCR + 1];   // +1: the z/4 planes start on different banks
    __shared__ int jmin_s, jmax_s;
    const int3 tile = xcd_tile<kXcdRunP>();
    const int4 bt = batches[tile.y];
    const int tb = threadIdx.x % kPB, tk = threadIdx.x / kPB;
    const int b = tile.x * kPB + tb;
    const int z0 = tile.z * ZC;
    const bool xmajor = bt.z != 0;
    const bool active = tk < bt.y && b < nb;
    const int a = order[bt.x + min(tk, bt.y - 1)];
    if (wg_on && !wg_on[((size_t)tile.y * gridDim.x + tile.x) * gridDim.z + tile.z]) {
        // none of this workgroup's rays is active: their outputs are zero
        if (active)
            for (int r = 0; r < NR; ++r) {
                T *dst = r == 0 ? sino_t + ((size_t)a * nb + b) * nz + z0
                                : sino_t + ((size_t)partner[a] * nb + (nb - 1 - b)) * nz + z0;
                for (int k = 0; k < ZC && z0 + k < nz; ++k) dst[k] = (T)0;
            }
        return;
    }
    const double2 tr = trig[a];
    const double sn = tr.x, cs = tr.y;
    // affine frame: s(m, j) = s00 + m dsm + j dsj, t(m, j) = t00 + m dtm + j dtj, u = (s + 1) inv_ds - 1/2
    const double c0 = centre(0, h);
    const double s00 = fma(-c0, sn, c0 * cs), t00 = fma(c0, cs, c0 * sn);
    const double dsj = (xmajor ? cs : -sn) * h, dsm = (xmajor ? -sn : cs) * h;
    const double dtj = (xmajor ? sn : cs) * h, dtm = (xmajor ? cs : sn) * h;
    const double du = dsj * inv_ds, dU = dsm * inv_ds, U00 = fma(s00 + 1.0, inv_ds, -0.5);
    const double inv_du = 1.0 / du;
    const T du_t = (T)du, dsj_t = (T)dsj, dtj_t = (T)dtj;
    const MarchF32 mc32 = march_f32(U00 - (double)b, dU, du, inv_du, s00, dsm, t00, dtm, nb);
    T acc[NR][ZC];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int k = 0; k < ZC; ++k) acc[r][k] = (T)0;
    const bool vec_ok = (nz & 3) == 0;
    for (int m0 = 0; m0 < n; m0 += kPCM) {
        if (threadIdx.x == 0) { jmin_s = 1 << 30; jmax_s = -(1 << 30); }
        __syncthreads();
        if (active) {
            double lo = 1e300, hi = -1e300;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const double U = fma((double)(e ? m0 + kPCM - 1 : m0), dU, U00);
                const double jA = ((double)b - 1.0 - U) * inv_du, jB = ((double)b + 1.0 - U) * inv_du;
                lo = fmin(lo, fmin(jA, jB));
                hi = fmax(hi, fmax(jA, jB));
            }
            atomicMin(&jmin_s, (int)floor(lo) - 1);
            atomicMax(&jmax_s, (int)ceil(hi) + 1);
        }
        __syncthreads();
        const int j0 = jmin_s;
        const int cr = min(jmax_s - j0 + 1, kPCR);
        const int mc = min(kPCM, n - m0);
        for (int e = threadIdx.x; e < mc * cr * Z4; e += 256) {
            const int z4 = e % Z4;
            const int rest = e / Z4;
            const int jj = rest % cr;
            const int mm = rest / cr;
            const int j = j0 + jj, m = m0 + mm;
            const int c = xmajor ? m : j, r = xmajor ? j : m;
            V4 v;
            T *vv = (T *)&v;
            if (j >= 0 && j < n && vial_ij(c, r, n)) {
                const T *src = vol_t + ((size_t)r * n + c) * nz + z0 + 4 * z4;
                if (vec_ok && z0 + 4 * z4 + 3 < nz) {
                    v = *(const V4 *)src;   // 16-byte aligned: nz % 4 == 0
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) vv[q] = (z0 + 4 * z4 + q < nz) ? src[q] : (T)0;
                }
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) vv[q] = (T)0;
            }
            lds[mm][z4][jj] = v;
        }
        __syncthreads();
        if (active) {
            for (int mm = 0; mm < mc; ++mm) {
                const int m = m0 + mm;
                int jlo;
                T d0, s0, t0;
                if constexpr (sizeof(T) == 4) {
                    jlo = march_step_f32(mc32, m, dsj_t, dtj_t, d0, s0, t0);
                } else {
                    const double U = fma((double)m, dU, U00);
                    const double jA = ((double)b - 1.0 - U) * inv_du, jB = ((double)b + 1.0 - U) * inv_du;
                    jlo = (int)ceil(fmin(jA, jB) - 1e-9);
                    const double jl = (double)jlo;
                    d0 = (T)(fma(jl, du, U) - (double)b);
                    s0 = (T)fma(jl, dsj, fma((double)m, dsm, s00));
                    t0 = (T)fma(jl, dtj, fma((double)m, dtm, t00));
                }
                const int jj0 = jlo - j0;
#pragma unroll
                for (int q = 0; q < NC; ++q) {
                    T hat = (T)1 - fabs(d0 + (T)q * du_t);
                    hat = hat > (T)0 ? hat : (T)0;
                    const T sq = s0 + (T)q * dsj_t;
                    T rr = (T)1 - sq * sq;
                    rr = rr > (T)0 ? sqrt_t<T>(rr) : (T)0;
                    const T tq = t0 + (T)q * dtj_t;
                    T w[NR];
                    w[0] = hat * exp_neg<T>(atten, tq + rr);
                    if (PAIR) w[NR - 1] = hat * exp_neg<T>(atten, rr - tq);
                    const int jj = min(max(jj0 + q, 0), cr - 1);
#pragma unroll
                    for (int z4 = 0; z4 < Z4; ++z4) {
                        const V4 v = lds[mm][z4][jj];
#pragma unroll
                        for (int r = 0; r < NR; ++r) {
                            acc[r][4 * z4 + 0] = fma(w[r], v.x, acc[r][4 * z4 + 0]);
                            acc[r][4 * z4 + 1] = fma(w[r], v.y, acc[r][4 * z4 + 1]);
                            acc[r][4 * z4 + 2] = fma(w[r], v.z, acc[r][4 * z4 + 2]);
                            acc[r][4 * z4 + 3] = fma(w[r], v.w, acc[r][4 * z4 + 3]);
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (!active) return;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        T *dst = r == 0 ? sino_t + ((size_t)a * nb + b) * nz + z0
                        : sino_t + ((size_t)partner[a] * nb + (nb - 1 - b)) * nz + z0;
#pragma unroll
        for (int z4 = 0; z4 < Z4; ++z4) {
            if (vec_ok && z0 + 4 * z4 + 3 < nz) {
                V4 v;
                v.x = acc[r][4 * z4 + 0]; v.y = acc[r][4 * z4 + 1]; v.z = acc[r][4 * z4 + 2]; v.w = acc[r][4 * z4 + 3];
                *(V4 *)(dst + 4 * z4) = v;
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (z0 + 4 * z4 + q < nz) dst[4 * z4 + q] = acc[r][4 * z4 + q];
            }
        }
    }
}

// ------------------------------------------------ 3D P, asynchronous staging
// Same rays, candidates and weights as project3d_kernel (FP32, nz % 4 == 0),
// but the volume strips are copied HBM -> LDS with direct-to-LDS loads
// (global_load_lds_dwordx4) into two buffers: while a workgroup computes the
// rays' contributions of one CM-step chunk from one buffer, the next chunk is
// already in flight into the other, so the staging latency is hidden behind
// compute instead of stalling every chunk.  CM = 1 halves the LDS footprint
// (more workgroups per CU) at one barrier per step; CM = 2 halves the
// barriers.
//
// LDS layout of a buffer: [step][z/4][kPCR + 1] 16-byte slots.  A wave's load
// instruction fills 64 consecutive slots, so each thread owns fixed slots
// (decoded once); per chunk only the source address changes.  Slots beyond a
// chunk's cross range, outside the grid or outside the vial load from a 16-byte
// zero block.  Cross ranges per (batch, bin group, step) come precomputed from
// the plan (conservative by one voxel on each side); a chunk stages the union
// of its steps' ranges.
constexpr int kDmaMaxCM = 2;
// s_waitcnt immediate (GFX9 encoding) that waits for at most n outstanding vector-memory
// operations and leaves the export and LDS/scalar counters unconstrained.
__host__ __device__ constexpr int vm_wait_imm(int n) {
    return (n & 0xF) | (((n >> 4) & 0x3) << 14) | (0x7 << 4) | (0xF << 8);
}

typedef __attribute__((address_space(3))) void lds_void;

// Workgroup barrier of the staging ring.  Each wave has already waited (vector-memory counter) for
// its own copies of the chunk it reads next, and its reads of earlier chunks have returned (LDS
// counter 0); copies of later chunks stay in flight.  A release fence would wait for those too,
// since staging copies write LDS; the empty asm statements keep the compiler from moving LDS
// accesses across the barrier instead.
constexpr int kLgkmWaitOnly = 0xF | (0x3 << 14) | (0x7 << 4);   // lgkmcnt(0), others unconstrained
__device__ __forceinline__ void ring_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(kLgkmWaitOnly);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

constexpr int kMaxListSteps = 1024;   // longest march that step lists serve
// A listed step's record, packed in 8 bytes: x = m | cross count << 10 | (first cross index + bias)
// << 17 (m < 1024, count <= kPCR < 128, 12 bits for the biased first index); y = vial interval of
// the step's grid line, lo | hi << 16.
constexpr int kListJ0Bias = 1024;
template <int ZC, int CM>
struct DmaRing {
    static constexpr int Z4 = ZC / 4, RS = kPCR + 1, SLOTS = CM * Z4 * RS, PER = (SLOTS + 255) / 256;
};

// One workgroup tile (bin group tile.x, view batch tile.y, z chunk x march split tile.z) of a
// grid of gx bin groups and gz z entries.  bufA..C and smeta are the kernel's LDS arrays.
template <int ZC, int NC, bool PAIR, bool SKIP, int CM, bool LIST, bool QUEUE>
__device__ __forceinline__ void p3d_dma_tile(
    const float *__restrict__ vol_t, float *__restrict__ sino_t, int n, int nz, int nb,
    const double2 *__restrict__ trig, const int *__restrict__ order, const int *__restrict__ partner,
    const int4 *__restrict__ batches, const int2 *__restrict__ ranges, const int2 *__restrict__ vial_rows,
    const float4 *__restrict__ zero16, double h, double inv_ds, float atten, const uint8_t *__restrict__ wg_on,
    int nsplit, long long split_stride, const PrimalFuse &fz, const int *__restrict__ step_list,
    const int *__restrict__ step_cnt, int3 tile, int gx, int gz, float4 *bufA, float4 *bufB, float4 *bufC,
    int2 *smeta) {
    static_assert(CM >= 1 && CM <= kDmaMaxCM, "chunk length");
    static_assert(!LIST || CM <= 2, "step lists walk one or two listed steps per chunk");
    constexpr int Z4 = DmaRing<ZC, CM>::Z4, RS = DmaRing<ZC, CM>::RS, SLOTS = DmaRing<ZC, CM>::SLOTS;
    constexpr int PER = DmaRing<ZC, CM>::PER;
    constexpr int NR = PAIR ? 2 : 1;
    const int tid = threadIdx.x;
    const int4 bt = batches[tile.y];
    // lane -> (bin, view): each wave holds two neighbouring views; a 16-lane quarter holds the same
    // 8 bins of both, whose candidate voxels nearly coincide, so one quarter's LDS reads stay
    // within about one pass of the 64 banks
    const int lane = tid & 63, wv = tid >> 6;
    const int tb = (lane & 7) | ((lane >> 4) << 3), tk = 2 * wv + ((lane >> 3) & 1);
    const int b = tile.x * kPB + tb;
    // grid.z = z chunks x march splits; split s walks its share of the chunks into partial sum s
    const int nzc = gz / nsplit, zb = tile.z % nzc, split = tile.z / nzc;
    const int z0 = zb * ZC;
    const bool xmajor = bt.z != 0;
    const bool active = tk < bt.y && b < nb;
    const int a = order[bt.x + min(tk, bt.y - 1)];
    if (wg_on && !wg_on[((size_t)tile.y * gx + tile.x) * nzc + zb]) {
        // none of this workgroup's rays is active: their outputs are zero (before any barrier);
        // with splits the reduction writes those zeros; with the fused primal step nothing changes
        if (active && nsplit == 1 && !fz.y)
            for (int r = 0; r < NR; ++r) {
                float4 *dst = (float4 *)(r == 0 ? sino_t + ((size_t)a * nb + b) * nz + z0
                                                : sino_t + ((size_t)partner[a] * nb + (nb - 1 - b)) * nz + z0);
                for (int z4 = 0; z4 < Z4 && z0 + 4 * z4 < nz; ++z4) dst[z4] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
        return;
    }
    const double2 tr = trig[a];
    const double sn = tr.x, cs = tr.y;
    const double c0 = centre(0, h);
    const double s00 = fma(-c0, sn, c0 * cs), t00 = fma(c0, cs, c0 * sn);
    const double dsj = (xmajor ? cs : -sn) * h, dsm = (xmajor ? -sn : cs) * h;
    const double dtj = (xmajor ? sn : cs) * h, dtm = (xmajor ? cs : sn) * h;
    const double du = dsj * inv_ds, dU = dsm * inv_ds, U00 = fma(s00 + 1.0, inv_ds, -0.5);
    const double inv_du = 1.0 / du;
    const float du_t = (float)du, dsj_t = (float)dsj, dtj_t = (float)dtj;
    const MarchF32 mc32 = march_f32(U00 - (double)b, dU, du, inv_du, s00, dsm, t00, dtm, nb);
    // the march: every step in chunks of CM, or (step lists) only the listed steps, in increasing
    // order and CM listed steps per chunk, each staged with its own cross range; the steps left out
    // stage nothing but zeros
    // LIST: each listed step's record (step, staged cross range, vial interval of its grid line) is
    // gathered into LDS first, so that a chunk's metadata costs one LDS read instead of a chain of
    // dependent scalar loads from global memory, and adds no vector-memory load to the staging waits
    // below (their counts cover the staging copies only)
    // (a static array of the kernel: the compiler then knows that the staging copies into the ring
    // never write it)
    const int2 *rg = ranges + ((size_t)tile.y * gx + tile.x) * n;
    int nch = (n + CM - 1) / CM, nlist = 0;
    if constexpr (LIST) {
        const size_t wgi = ((size_t)tile.y * gx + tile.x) * nzc + zb;
        nlist = __builtin_amdgcn_readfirstlane(step_cnt[wgi]);
        nch = (nlist + CM - 1) / CM;   // a chunk: CM consecutive entries of the list
        for (int i = tid; i < nlist; i += 256) {
            const int m = step_list[wgi * n + i];
            const int2 r = rg[m], v = vial_rows[m];
            smeta[i] = make_int2(m | (r.y << 10) | ((r.x + kListJ0Bias) << 17), (v.x & 0xFFFF) | (v.y << 16));
        }
        __syncthreads();
    }
    auto first_step = [&](int k) { return __builtin_amdgcn_readfirstlane(k * CM); };
    // LIST: entry e of the list (uniform): step m, staged cross range r (first index, count) and the
    // vial interval v of its grid line; entries past the list stage and compute nothing
    auto list_rec = [&](int e, int &m, int2 &r, int2 &v) {
        if (e < nlist) {
            const int2 sm = smeta[e];
            const int ex = __builtin_amdgcn_readfirstlane(sm.x), ey = __builtin_amdgcn_readfirstlane(sm.y);
            m = ex & 1023;
            r = make_int2((ex >> 17) - kListJ0Bias, (ex >> 10) & 127);
            v = make_int2(ey & 0xFFFF, ey >> 16);
        } else {
            m = 0;
            r = make_int2(0, 0);
            v = make_int2(1, 0);
        }
    };
    const size_t zrow = (size_t)(nz >> 2), zoff = (size_t)(z0 >> 2);
    const float4 *vol4 = (const float4 *)vol_t;

    // staged cross range of chunk k: the union of its steps' ranges (first index, count)
    auto chunk_range = [&](int k) {
        const int m0 = first_step(k);   // uniform: scalar loads
        int lo = rg[m0].x, hi = rg[m0].x + rg[m0].y;
#pragma unroll
        for (int q = 1; q < CM; ++q)
            if (m0 + q < n) {
                const int2 r = rg[m0 + q];
                lo = min(lo, r.x);
                hi = max(hi, r.x + r.y);
            }
        return make_int2(lo, hi - lo);
    };

    // fixed slots of this thread: (step, z/4, cross offset)
    int s_mm[PER], s_z4[PER], s_jj[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int slot = i * 256 + tid;
        s_mm[i] = slot / (Z4 * RS);
        const int rem = slot - s_mm[i] * (Z4 * RS);
        s_z4[i] = rem / RS;
        s_jj[i] = rem - s_z4[i] * RS;
    }
    auto issue = [&](float4 *buf, int k) {
        // per row of the chunk (uniform): step, staged cross range and vial interval; without step
        // lists the rows are consecutive steps sharing the union of their ranges
        int mq[CM];
        int2 rq[CM], vq[CM];
        if constexpr (LIST) {
#pragma unroll
            for (int q = 0; q < CM; ++q) list_rec(k * CM + q, mq[q], rq[q], vq[q]);
        } else {
            const int2 r = chunk_range(k);
            const int m0 = first_step(k);
#pragma unroll
            for (int q = 0; q < CM; ++q) {
                mq[q] = m0 + q;
                rq[q] = r;
                vq[q] = vial_rows[min(m0 + q, n - 1)];
            }
        }
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            if (i * 256 + tid < SLOTS) {
                const int mm = CM == 1 ? 0 : s_mm[i];
                int m = mq[0];
                int2 r = rq[0], v = vq[0];
#pragma unroll
                for (int q = 1; q < CM; ++q)
                    if (mm == q) { m = mq[q]; r = rq[q]; v = vq[q]; }
                const int j = r.x + s_jj[i];
                const float4 *src = zero16;
                if (m < n && s_jj[i] < r.y && z0 + 4 * s_z4[i] < nz && j >= v.x && j <= v.y)
                    src = vol4 + (xmajor ? ((size_t)j * n + m) : ((size_t)m * n + j)) * zrow + zoff + s_z4[i];
                __builtin_amdgcn_global_load_lds((const void *)src, (lds_void *)(buf + i * 256 + (tid & ~63)), 16, 0,
                                                 0);
            }
        }
        asm volatile("" ::: "memory");   // keep the copies ahead of the compute that follows
    };

    float acc[NR][ZC];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int k = 0; k < ZC; ++k) acc[r][k] = 0.f;

    auto compute = [&](const float4 *buf, int k) {
        int2 r = make_int2(0, 0);
        int m0 = 0, mc = CM;
        if constexpr (!LIST) {
            r = chunk_range(k);
            m0 = first_step(k);
            mc = min(CM, n - m0);
        }
        for (int mm = 0; mm < mc; ++mm) {
            int m = m0 + mm;
            if constexpr (LIST) {
                if (k * CM + mm >= nlist) break;   // the list's last chunk may be short
                int2 v;
                list_rec(k * CM + mm, m, r, v);
            }
            const int j0 = r.x, cr = r.y;
            float d0, s0, t0;
            const int jlo = march_step_f32(mc32, m, dsj_t, dtj_t, d0, s0, t0);
            const int jj0 = jlo - j0;
            const float4 *row = buf + mm * (Z4 * RS);
#pragma unroll
            for (int q = 0; q < NC; ++q) {
                float hat = 1.f - fabsf(d0 + (float)q * du_t);
                hat = hat > 0.f ? hat : 0.f;
                const float sq = s0 + (float)q * dsj_t;
                float rr = 1.f - sq * sq;
                rr = rr > 0.f ? sqrt_t<float>(rr) : 0.f;
                const float tq = t0 + (float)q * dtj_t;
                float w[NR];
                w[0] = hat * exp_neg<float>(atten, tq + rr);
                if (PAIR) w[NR - 1] = hat * exp_neg<float>(atten, rr - tq);
                const int jj = min(max(jj0 + q, 0), cr - 1);
                // SKIP: lanes whose candidate lies outside their ray's reach issue no LDS reads
                if (SKIP && !(hat > 0.f)) continue;
                // all of the candidate's LDS reads go out before its FMAs, so their latencies
                // overlap instead of being waited out two reads at a time
                float4 v[Z4];
#pragma unroll
                for (int z4 = 0; z4 < Z4; ++z4) v[z4] = row[z4 * RS + jj];
                __builtin_amdgcn_sched_barrier(0);   // keep the reads ahead of the FMAs below
#pragma unroll
                for (int z4 = 0; z4 < Z4; ++z4) {
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        acc[r][4 * z4 + 0] = fmaf(w[r], v[z4].x, acc[r][4 * z4 + 0]);
                        acc[r][4 * z4 + 1] = fmaf(w[r], v[z4].y, acc[r][4 * z4 + 1]);
                        acc[r][4 * z4 + 2] = fmaf(w[r], v[z4].z, acc[r][4 * z4 + 2]);
                        acc[r][4 * z4 + 3] = fmaf(w[r], v[z4].w, acc[r][4 * z4 + 3]);
                    }
                }
            }
        }
    };

    // Ring of three buffers: chunk k + 2 is copied while chunk k is consumed, so each copy has two
    // chunks of compute to land.  Before consuming chunk k a wave waits until its own copies of
    // chunk k have landed (vector-memory counter: the copies of chunk k + 1 may stay in flight;
    // loads retire in order), then the barrier makes that hold for all waves and frees the buffer
    // the next copy goes to.  A wave issues PER copies per chunk, or PER - 1 when its lanes have no
    // slot in the last copy round (that copy is branched around).
    const bool full_wave = (PER - 1) * 256 + 64 * __builtin_amdgcn_readfirstlane(tid >> 6) < SLOTS;
    constexpr int kWaitFull = vm_wait_imm(PER), kWaitPart = vm_wait_imm(PER - 1);
    const int per = (nch + nsplit - 1) / nsplit, kb = split * per, ke = min(nch, kb + per);
    auto step = [&](const float4 *cur, float4 *next2, int k) {
        if (k + 1 < ke) {
            if (full_wave) __builtin_amdgcn_s_waitcnt(kWaitFull);
            else __builtin_amdgcn_s_waitcnt(kWaitPart);
        } else {
            __builtin_amdgcn_s_waitcnt(0);
        }
        ring_barrier();
        if (k + 2 < ke) issue(next2, k + 2);
        if (active) compute(cur, k);
    };
    if (kb < ke) issue(bufA, kb);
    if (kb + 1 < ke) issue(bufB, kb + 1);
    for (int k = kb; k < ke; k += 3) {
        step(bufA, bufC, k);
        if (k + 1 >= ke) break;
        step(bufB, bufA, k + 1);
        if (k + 2 >= ke) break;
        step(bufC, bufB, k + 2);
    }
    if (!active) return;
    if (fz.y) {
        // fused primal step on this lane's rays (same arithmetic as the solver's primal kernel)
        const float tf = (float)*fz.tau_fac, w = (float)fz.w_rho[0], rho = (float)fz.w_rho[1];
        if constexpr (QUEUE) {
            // in the work queue the epilogue's memory waits lie on the workgroup's path to its next
            // tile, so its loads go out in batches: every ray's activity words first, then y, T_j
            // and y0 of four four-slice groups at once (groups without an active ray read a zero
            // block), a few waits per tile instead of one or two per group
            size_t base[NR];
            uint32_t am[NR][Z4];
    #pragma unroll
            for (int r = 0; r < NR; ++r) {
                base[r] = r == 0 ? ((size_t)a * nb + b) * nz + z0 : ((size_t)partner[a] * nb + (nb - 1 - b)) * nz + z0;
    #pragma unroll
                for (int z4 = 0; z4 < Z4; ++z4)
                    am[r][z4] = z0 + 4 * z4 < nz ? *(const uint32_t *)(fz.act + base[r] + 4 * z4) : 0u;
            }
    #pragma unroll
            for (int r = 0; r < NR; ++r) {
    #pragma unroll
                for (int h = 0; h < Z4; h += 4) {
                    constexpr int G = Z4 < 4 ? Z4 : 4;
                    float4 yo[G], tj[G], a0[G];
    #pragma unroll
                    for (int g = 0; g < G; ++g) {
                        const size_t i = base[r] + 4 * (h + g);
                        const bool on = am[r][h + g] != 0u;
                        yo[g] = on ? *(const float4 *)(fz.y + i) : *zero16;
                        tj[g] = on ? *(const float4 *)(fz.Tj + i) : *zero16;
                        a0[g] = on ? *(const float4 *)(fz.y0 + i) : *zero16;
                    }
    #pragma unroll
                    for (int g = 0; g < G; ++g) {
                        const uint32_t m = am[r][h + g];
                        if (!m) continue;
                        const size_t i = base[r] + 4 * (h + g);
                        const float yv[4] = {yo[g].x, yo[g].y, yo[g].z, yo[g].w}, tv[4] = {tj[g].x, tj[g].y, tj[g].z, tj[g].w},
                                    av[4] = {a0[g].x, a0[g].y, a0[g].z, a0[g].w};
                        float t4[4], y4[4];
    #pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            float v = yv[k] - tf * tv[k] * acc[r][4 * (h + g) + k];
                            v = v > 0.f ? v : 0.f;
                            t4[k] = v;
                            y4[k] = w * ((1.f + rho) * v - rho * yv[k]) + (1.f - w) * av[k];
                        }
                        if (((m - 0x01010101u) & ~m & 0x80808080u) == 0) {   // all four active
                            *(float4 *)(fz.yt + i) = make_float4(t4[0], t4[1], t4[2], t4[3]);
                            *(float4 *)(fz.y + i) = make_float4(y4[0], y4[1], y4[2], y4[3]);
                        } else {
    #pragma unroll
                            for (int k = 0; k < 4; ++k)
                                if ((m >> (8 * k)) & 0xFFu) { fz.yt[i + k] = t4[k]; fz.y[i + k] = y4[k]; }
                        }
                    }
                    // one batch of loads live at a time: the next batch is not hoisted above this one
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const size_t base = r == 0 ? ((size_t)a * nb + b) * nz + z0
                                           : ((size_t)partner[a] * nb + (nb - 1 - b)) * nz + z0;
#pragma unroll
                for (int z4 = 0; z4 < Z4; ++z4) {
                    const size_t i = base + 4 * z4;
                    if (z0 + 4 * z4 >= nz) continue;
                    const uint32_t m = *(const uint32_t *)(fz.act + i);
                    if (!m) continue;
                    const float4 yo = *(const float4 *)(fz.y + i), tj = *(const float4 *)(fz.Tj + i),
                                 a0 = *(const float4 *)(fz.y0 + i);
                    const float yv[4] = {yo.x, yo.y, yo.z, yo.w}, tv[4] = {tj.x, tj.y, tj.z, tj.w},
                                av[4] = {a0.x, a0.y, a0.z, a0.w};
                    float t4[4], y4[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        float v = yv[k] - tf * tv[k] * acc[r][4 * z4 + k];
                        v = v > 0.f ? v : 0.f;
                        t4[k] = v;
                        y4[k] = w * ((1.f + rho) * v - rho * yv[k]) + (1.f - w) * av[k];
                    }
                    if (((m - 0x01010101u) & ~m & 0x80808080u) == 0) {   // all four active
                        *(float4 *)(fz.yt + i) = make_float4(t4[0], t4[1], t4[2], t4[3]);
                        *(float4 *)(fz.y + i) = make_float4(y4[0], y4[1], y4[2], y4[3]);
                    } else {
#pragma unroll
                        for (int k = 0; k < 4; ++k)
                            if ((m >> (8 * k)) & 0xFFu) { fz.yt[i + k] = t4[k]; fz.y[i + k] = y4[k]; }
                    }
                }
            }
        }
        return;
    }
    float *out = sino_t + (size_t)split * split_stride;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        float *dst = r == 0 ? out + ((size_t)a * nb + b) * nz + z0
                            : out + ((size_t)partner[a] * nb + (nb - 1 - b)) * nz + z0;
#pragma unroll
        for (int z4 = 0; z4 < Z4; ++z4) {
            if (z0 + 4 * z4 < nz) {
                float4 v;
                v.x = acc[r][4 * z4 + 0]; v.y = acc[r][4 * z4 + 1]; v.z = acc[r][4 * z4 + 2]; v.w = acc[r][4 * z4 + 3];
                *(float4 *)(dst + 4 * z4) = v;
            }
        }
    }
}

// Grid mode (!QUEUE): one workgroup per tile of the launch grid.  Work-queue mode (QUEUE, step
// lists of an LP solve): a persistent grid takes tiles from items[0, n_items) in that order -- the
// switched-on tiles, longest step list first -- through an atomic counter, so the chip stays evenly
// loaded while the tiles' walks differ several-fold in length; tile indices are flag indices of a
// virtual grid of gx bin groups x batches x gz z chunks (no march splits).  queue[0] counts taken
// tiles, queue[1] finished workgroups; the last workgroup to finish sets both back to zero, so
// consecutive launches on one stream reuse the counters (they start zeroed).
template <int ZC, int NC, bool PAIR, bool SKIP, int CM, bool LIST, bool QUEUE>
__global__ void __launch_bounds__(256) project3d_dma_kernel(
    const float *__restrict__ vol_t, float *__restrict__ sino_t, int n, int nz, int nb,
    const double2 *__restrict__ trig, const int *__restrict__ order, const int *__restrict__ partner,
    const int4 *__restrict__ batches, const int2 *__restrict__ ranges, const int2 *__restrict__ vial_rows,
    const float4 *__restrict__ zero16, double h, double inv_ds, float atten, const uint8_t *__restrict__ wg_on,
    int nsplit, long long split_stride, PrimalFuse fz, const int *__restrict__ step_list,
    const int *__restrict__ step_cnt, const int *__restrict__ items, int n_items, int *__restrict__ queue, int vgx,
    int vgz) {
    constexpr int SLOTS = DmaRing<ZC, CM>::SLOTS;
    // three separate arrays, not one indexed ring: the compiler tells LDS variables apart when it
    // decides which staging copies a read has to wait for, but not slices of one array
    __shared__ float4 bufA[SLOTS];
    __shared__ float4 bufB[SLOTS];
    __shared__ float4 bufC[SLOTS];
    __shared__ int2 smeta[LIST ? kMaxListSteps : 1];
    if constexpr (!QUEUE) {
        p3d_dma_tile<ZC, NC, PAIR, SKIP, CM, LIST, false>(vol_t, sino_t, n, nz, nb, trig, order, partner, batches,
                                                         ranges, vial_rows, zero16, h, inv_ds, atten, wg_on, nsplit,
                                                         split_stride, fz, step_list, step_cnt, xcd_tile<kXcdRunP>(),
                                                         gridDim.x, gridDim.z, bufA, bufB, bufC, smeta);
        return;
    }
    static_assert(!QUEUE || LIST, "the work queue serves listed marches");
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
        __syncthreads();
        const int it = s_item;
        __syncthreads();   // every wave has its tile before thread 0 takes the next one
        if (it >= n_items) break;
        const int wgi = items[it];
        const int zb = wgi % vgz, t = wgi / vgz;
        p3d_dma_tile<ZC, NC, PAIR, SKIP, CM, LIST, QUEUE>(vol_t, sino_t, n, nz, nb, trig, order, partner, batches,
                                                         ranges, vial_rows, zero16, h, inv_ds, atten, wg_on, 1,
                                                         split_stride, fz, step_list, step_cnt,
                                                         make_int3(t % vgx, t / vgx, zb), vgx, vgz, bufA, bufB, bufC,
                                                         smeta);
        __syncthreads();   // the tile's LDS reads are done before the next tile stages into the ring
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(queue + 1, 1) == (int)gridDim.x - 1) {   // every workgroup has taken its last tile
            atomicExch(queue, 0);
            atomicExch(queue + 1, 0);
        }
    }
}

// Batched transpose: [B][R][C] -> [B][C][R] (out = in^T, or out += in^T).
template <typename T>
__global__ void __launch_bounds__(256) transpose_kernel(const T *__restrict__ in, T *__restrict__ out, int rows,
                                                        int cols, int accumulate) {
    __shared__ T tile[64][65];
    const size_t plane = (size_t)rows * cols;
    const T *src = in + (size_t)blockIdx.z * plane;
    T *dst = out + (size_t)blockIdx.z * plane;
    const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {
        const int r = r0 + i, c = c0 + tx;
        tile[i][tx] = (r < rows && c < cols) ? src[(size_t)r * cols + c] : (T)0;
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const int c = c0 + i, r = r0 + tx;
        if (r < rows && c < cols) {
            const size_t o = (size_t)c * rows + r;
            dst[o] = accumulate ? dst[o] + tile[tx][i] : tile[tx][i];
        }
    }
}

// Flagged variant for masked solves, in tiles of kTrRows rows x kTrCols columns (one plane): tiles
// that are off are not written.  Reads are 1 KB rows; a column's kTrRows values are written as one
// 64-byte run.
static_assert(kTrCols == 256 && 256 % kTrRows == 0, "one column per thread when reading a tile row");

template <typename T>
__global__ void __launch_bounds__(256) transpose_flagged_kernel(const T *__restrict__ in, T *__restrict__ out,
                                                                int rows, int cols,
                                                                const uint8_t *__restrict__ tile_on) {
    __shared__ T tile[kTrRows][kTrCols + 1];
    if (!tile_on[(size_t)blockIdx.y * gridDim.x + blockIdx.x]) return;
    const int c0 = blockIdx.x * kTrCols, r0 = blockIdx.y * kTrRows, t = threadIdx.x;
    // all kTrRows loads of a thread in flight at once: unconditional, from a clamped address, with the
    // values outside the matrix zeroed as they are written to LDS
    const int cl = min(c0 + t, cols - 1);
    T v[kTrRows];
#pragma unroll
    for (int i = 0; i < kTrRows; ++i) v[i] = in[(size_t)min(r0 + i, rows - 1) * cols + cl];
#pragma unroll
    for (int i = 0; i < kTrRows; ++i) tile[i][t] = (r0 + i < rows && c0 + t < cols) ? v[i] : (T)0;
    __syncthreads();
    const int rr = t % kTrRows, r = r0 + rr;
#pragma unroll
    for (int k = 0; k < kTrCols / (256 / kTrRows); ++k) {
        const int cc = t / kTrRows + (256 / kTrRows) * k, c = c0 + cc;
        if (r < rows && c < cols) out[(size_t)c * rows + r] = tile[rr][cc];
    }
}

template <typename T>
static void transpose(const void *in, void *out, int batch, int rows, int cols, int accumulate, hipStream_t s,
                      const uint8_t *tile_on = nullptr) {
    if (tile_on) {   // one plane, overwrite
        const dim3 grid((cols + kTrCols - 1) / kTrCols, (rows + kTrRows - 1) / kTrRows, 1);
        hipLaunchKernelGGL((transpose_flagged_kernel<T>), grid, dim3(256), 0, s, (const T *)in, (T *)out, rows, cols,
                           tile_on);
        return;
    }
    const dim3 grid((cols + 63) / 64, (rows + 63) / 64, batch);
    hipLaunchKernelGGL((transpose_kernel<T>), grid, dim3(256), 0, s, (const T *)in, (T *)out, rows, cols, accumulate);
}

static int transpose_any(sipo_plan p, const void *in, void *out, int batch, int rows, int cols, int accumulate,
                         hipStream_t s, const uint8_t *tile_on = nullptr) {
    if (p->dtype == SIPO_F64) transpose<double>(in, out, batch, rows, cols, accumulate, s, tile_on);
    else transpose<float>(in, out, batch, rows, cols, accumulate, s, tile_on);
    SIPO_LAUNCHED("transpose_kernel");
    return SIPO_OK;
}

// --------------------------------------------------------- host: batching
// Staged cross range (first index j0 and count, with the kernels' one-voxel
// guards) of a bundle of views and the kPB bins from b0 over steps m0 .. m1.
static void staged_range(bool xmajor, const double2 *trig, const int *idx, int cnt, int b0, int m0, int m1, double h,
                         double inv_ds, int *j0, int *count) {
    double lo = 1e300, hi = -1e300;
    for (int k = 0; k < cnt; ++k) {
        const double sn = trig[idx[k]].x, cs = trig[idx[k]].y;
        for (int e = 0; e < 2; ++e) {
            const int m = e ? m1 : m0;
            const double c0 = -1.0 + 0.5 * h, pm = -1.0 + (m + 0.5) * h;
            const double s0 = xmajor ? -pm * sn + c0 * cs : -c0 * sn + pm * cs;
            const double U = (s0 + 1.0) * inv_ds - 0.5;
            const double du = (xmajor ? cs : -sn) * h * inv_ds;
            for (int f = 0; f < 2; ++f) {
                const double j = ((f ? b0 + kPB : b0 - 1.0) - U) / du;
                lo = std::min(lo, j);
                hi = std::max(hi, j);
            }
        }
    }
    *j0 = (int)std::floor(lo) - 1;
    *count = (int)std::ceil(hi) + 1 - *j0 + 1;
}

// Cross-axis range (in voxels, with the kernel's guards) a bundle of views and
// kPB bins starting at b0 can reach during the kPCM steps starting at m0.
static int chunk_range(bool xmajor, const double2 *trig, const int *idx, int cnt, int b0, int m0, double h,
                       double inv_ds) {
    int j0, count;
    staged_range(xmajor, trig, idx, cnt, b0, m0, m0 + kPCM - 1, h, inv_ds, &j0, &count);
    return count;
}

// Opposite view of every view (sin and cos both change sign, to 1e-12), or -1;
// views are paired greedily, each at most once.
static std::vector<int> opposite_views(const double2 *trig, int na) {
    std::vector<int> idx(na), opp(na, -1);
    for (int a = 0; a < na; ++a) idx[a] = a;
    std::sort(idx.begin(), idx.end(), [&](int i, int j) {
        return trig[i].x < trig[j].x || (trig[i].x == trig[j].x && trig[i].y < trig[j].y);
    });
    constexpr double eps = 1e-12;
    for (int a = 0; a < na; ++a) {
        if (opp[a] >= 0) continue;
        const double ts = -trig[a].x, tc = -trig[a].y;
        auto it = std::lower_bound(idx.begin(), idx.end(), ts - eps,
                                   [&](int i, double v) { return trig[i].x < v; });
        for (; it != idx.end() && trig[*it].x <= ts + eps; ++it) {
            const int b = *it;
            if (b != a && opp[b] < 0 && std::fabs(trig[b].y - tc) <= eps) {
                opp[a] = b;
                opp[b] = a;
                break;
            }
        }
    }
    return opp;
}

int plan_build_batches(sipo_plan p, const double2 *trig) {
    const double h = 2.0 / p->n, inv_ds = 0.5 * p->n_bins;
    const std::vector<int> opp = opposite_views(trig, p->n_angles);
    bool pair = p->n_angles >= 2;
    for (int a = 0; a < p->n_angles; ++a) pair = pair && opp[a] >= 0;
    auto walked = [&](int a) { return !pair || a < opp[a]; };
    std::vector<int> order;
    double min_du = 1e300;
    for (int a = 0; a < p->n_angles; ++a)
        if (walked(a) && std::fabs(trig[a].y) >= std::fabs(trig[a].x)) order.push_back(a);
    const int nx = (int)order.size();
    for (int a = 0; a < p->n_angles; ++a)
        if (walked(a) && !(std::fabs(trig[a].y) >= std::fabs(trig[a].x))) order.push_back(a);
    const int nw = (int)order.size();
    for (int k = 0; k < nw; ++k) {
        const double sn = trig[order[k]].x, cs = trig[order[k]].y;
        min_du = std::min(min_du, std::fabs((k < nx ? cs : -sn) * h * inv_ds));
    }
    std::vector<int4> batches;
    bool ok = true;
    const int last_b0 = ((p->n_bins - 1) / kPB) * kPB;
    const int last_m0 = ((p->n - 1) / kPCM) * kPCM;
    auto fits = [&](bool xm, int start, int cnt) {
        int worst = 0;
        for (int b0 : {0, last_b0})
            for (int m0 : {0, last_m0})
                worst = std::max(worst, chunk_range(xm, trig, order.data() + start, cnt, b0, m0, h, inv_ds));
        return worst + 2 <= kPCR;
    };
    for (int part = 0; part < 2; ++part) {
        const int beg = part ? nx : 0, end = part ? nw : nx;
        int i = beg;
        while (i < end) {
            int cnt = 1;
            if (!fits(part == 0, i, 1)) ok = false;
            while (cnt < kPV && i + cnt < end && fits(part == 0, i, cnt + 1)) ++cnt;
            batches.push_back(make_int4(i, cnt, part == 0 ? 1 : 0, 0));
            i += cnt;
        }
    }
    // candidates per ray step: the integers in an interval of length 2/|du| (plus guards)
    const int nc = (int)std::floor(2.0 / min_du + 1e-6) + 1;
    p->p3d_nc = nc <= 3 ? 3 : (nc <= 4 ? 4 : (nc <= 6 ? 6 : 0));
    p->p3d_pair = pair;
    p->n_walk = nw;
    p->p3d_zc = p->dtype == SIPO_F64 ? 16 : 32;
    p->p3d_skip = false;
    p->p3d_cm = kDmaMaxCM;
    p->bp3d_zc = p->dtype == SIPO_F64 ? 16 : 32;
    p->blur_zc = 0;
    p->n_batches = (int)batches.size();
    p->p3d_ok = ok && p->p3d_nc > 0;
    p->bp3d_ok = bp3d_fits(p->n, p->n_bins);
    // staged cross range of every (batch, bin group, step) for the asynchronous projector; its chunks
    // of up to kDmaMaxCM steps stage the union of their steps' ranges, which must fit kPCR
    const int ngroups = (p->n_bins + kPB - 1) / kPB;
    std::vector<int2> ranges;
    bool dma = p->dtype == SIPO_F32 && (p->nz & 3) == 0 && p->p3d_ok;
    int j0_min = 0, j0_max = 0;
    if (dma) {
        ranges.resize((size_t)batches.size() * ngroups * p->n);
        for (size_t bi = 0; bi < batches.size() && dma; ++bi) {
            const int4 bt = batches[bi];
            for (int g = 0; g < ngroups && dma; ++g) {
                int2 *row = ranges.data() + (bi * ngroups + g) * p->n;
                for (int m = 0; m < p->n; ++m) {
                    int j0, cr;
                    staged_range(bt.z != 0, trig, order.data() + bt.x, bt.y, g * kPB, m, m, h, inv_ds, &j0, &cr);
                    row[m] = make_int2(j0, cr);
                    j0_min = std::min(j0_min, j0);
                    j0_max = std::max(j0_max, j0);
                }
                for (int m0 = 0; m0 < p->n && dma; m0 += kDmaMaxCM) {
                    int lo = row[m0].x, hi = row[m0].x + row[m0].y;
                    for (int q = 1; q < kDmaMaxCM && m0 + q < p->n; ++q) {
                        lo = std::min(lo, row[m0 + q].x);
                        hi = std::max(hi, row[m0 + q].x + row[m0 + q].y);
                    }
                    if (hi - lo > kPCR) dma = false;
                }
            }
        }
    }
    std::vector<int2> vial(p->n);
    for (int m = 0; m < p->n; ++m) {
        // indices j with (2j+1-n)^2 <= n^2 - (2m+1-n)^2, found from a square root and fixed up exactly
        const long long nn = p->n, am = 2LL * m + 1 - nn, rem = nn * nn - am * am;
        long long c = (long long)std::sqrt((double)rem);
        while (c > 0 && c * c > rem) --c;
        while ((c + 1) * (c + 1) <= rem) ++c;
        long long lo = (nn - 1 - c + 1) / 2, hi = (nn - 1 + c) / 2;   // ceil((n-1-c)/2), floor((n-1+c)/2)
        if (nn - 1 - c < 0) lo = 0;
        auto inside = [&](long long j) { const long long q = 2 * j + 1 - nn; return q * q <= rem; };
        while (lo <= hi && !inside(lo)) ++lo;
        while (hi >= lo && !inside(hi)) --hi;
        vial[m] = lo <= hi ? make_int2((int)lo, (int)hi) : make_int2(1, 0);
    }
    p->p3d_dma_ok = p->p3d_dma = dma;
    p->p3d_list_ok = dma && p->n <= kMaxListSteps && j0_min >= -kListJ0Bias && j0_max < (1 << 12) - kListJ0Bias;
    if (dma) {
        SIPO_TRY(plan_alloc(p, (void **)&p->d_ranges, sizeof(int2) * ranges.size()));
        SIPO_HIP(hipMemcpy(p->d_ranges, ranges.data(), sizeof(int2) * ranges.size(), hipMemcpyHostToDevice));
    }
    SIPO_TRY(plan_alloc(p, (void **)&p->d_vial_rows, sizeof(int2) * vial.size()));
    SIPO_HIP(hipMemcpy(p->d_vial_rows, vial.data(), sizeof(int2) * vial.size(), hipMemcpyHostToDevice));
    SIPO_TRY(plan_alloc(p, (void **)&p->d_zero, 256));

    SIPO_HIP(hipMemset(p->d_zero, 0, 256));
    // batch of every view (2 * batch, plus 1 for the opposite view of a walked one), -1 if unwalked
    std::vector<int> vbatch(p->n_angles, -1);
    for (size_t bi = 0; bi < batches.size(); ++bi)
        for (int k = batches[bi].x; k < batches[bi].x + batches[bi].y; ++k) {
            const int v = order[k];
            vbatch[v] = 2 * (int)bi;
            if (pair && opp[v] >= 0) vbatch[opp[v]] = 2 * (int)bi + 1;
        }
    SIPO_TRY(plan_alloc(p, (void **)&p->d_view_batch, sizeof(int) * p->n_angles));
    SIPO_HIP(hipMemcpy(p->d_view_batch, vbatch.data(), sizeof(int) * p->n_angles, hipMemcpyHostToDevice));
    SIPO_TRY(plan_alloc(p, (void **)&p->d_batches, sizeof(int4) * std::max<size_t>(batches.size(), 1)));
    SIPO_TRY(plan_alloc(p, (void **)&p->d_partner, sizeof(int) * p->n_angles));
    if (!batches.empty())
        SIPO_HIP(hipMemcpy(p->d_batches, batches.data(), sizeof(int4) * batches.size(), hipMemcpyHostToDevice));
    SIPO_HIP(hipMemcpy(p->d_angle_order, order.data(), sizeof(int) * order.size(), hipMemcpyHostToDevice));
    SIPO_HIP(hipMemcpy(p->d_partner, opp.data(), sizeof(int) * opp.size(), hipMemcpyHostToDevice));
    return SIPO_OK;
}

// ------------------------------------------------------------------ launchers
template <typename T>
static int bp_slices(sipo_plan p, const void *sino, void *vol, int accumulate, hipStream_t s) {
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
static int fp_slices(sipo_plan p, const void *vol, void *sino, int accumulate, hipStream_t s) {
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

template <typename T, int ZC>
static void bp3d_zc(sipo_plan p, const void *sino_t, void *vol, int accumulate, hipStream_t s, const uint8_t *on,
                    const SplitSpec &sp) {
    const double h = 2.0 / p->n, inv_ds = 0.5 * p->n_bins;
    const int ns = (sp.parts > 1 && !accumulate) ? sp.parts : 1;
    const int gx = (p->n + kBpTX - 1) / kBpTX, gy = (p->n + kBpTY - 1) / kBpTY, gz = (p->nz + ZC - 1) / ZC;
    if (p->nz % 4 == 0 && ZC <= 16)
        hipLaunchKernelGGL((backproject3d_kernel<T, ZC, ZC <= 16>), dim3(gx, gy, gz * ns), dim3(256), 0, s,
                           (const T *)sino_t, (T *)(ns > 1 ? sp.partial : vol), p->n, p->nz, p->n_angles, p->n_bins,
                           p->d_trig, h, inv_ds, (T)p->atten, accumulate, on, ns, (long long)p->vol_elems(),
                           on ? sp.need : nullptr);
    else
        hipLaunchKernelGGL((backproject3d_kernel<T, ZC, false>), dim3(gx, gy, gz * ns), dim3(256), 0, s,
                           (const T *)sino_t, (T *)(ns > 1 ? sp.partial : vol), p->n, p->nz, p->n_angles, p->n_bins,
                           p->d_trig, h, inv_ds, (T)p->atten, accumulate, on, ns, (long long)p->vol_elems(),
                           on ? sp.need : nullptr);
    if (ns > 1) {
        const long long total = (long long)p->vol_elems();
        hipLaunchKernelGGL((k_bp3d_reduce<T, ZC>), dim3(gx, gy, gz), dim3(256), 0, s, (const T *)sp.partial,
                           (T *)vol, on, p->n, p->nz, ns, total, sp.keep_off ? 1 : 0);
    }
}

template <typename T>
static int bp3d(sipo_plan p, const void *sino_t, void *vol, int accumulate, hipStream_t s, const uint8_t *on,
                const SplitSpec &sp) {
    switch (p->bp3d_zc) {
        case 4: bp3d_zc<T, 4>(p, sino_t, vol, accumulate, s, on, sp); break;
        case 8: bp3d_zc<T, 8>(p, sino_t, vol, accumulate, s, on, sp); break;
        case 16: bp3d_zc<T, 16>(p, sino_t, vol, accumulate, s, on, sp); break;
        case 32:
            if constexpr (sizeof(T) == 4) { bp3d_zc<T, 32>(p, sino_t, vol, accumulate, s, on, sp); break; }
            else return fail(SIPO_E_UNSUPPORTED, "3D backprojector: 32 slices per thread in FP64");
        default: return fail(SIPO_E_UNSUPPORTED, "3D backprojector: %d slices per thread", p->bp3d_zc);
    }
    SIPO_LAUNCHED("backproject3d_kernel");
    return SIPO_OK;
}

template <typename T, int ZC, int NC>
static void fp3d_nc(sipo_plan p, const void *vol_t, void *sino_t, hipStream_t s, const uint8_t *on) {
    const double h = 2.0 / p->n, inv_ds = 0.5 * p->n_bins;
    const dim3 grid((p->n_bins + kPB - 1) / kPB, p->n_batches, (p->nz + ZC - 1) / ZC);
    if (p->p3d_pair)
        hipLaunchKernelGGL((project3d_kernel<T, ZC, NC, true>), grid, dim3(256), 0, s, (const T *)vol_t, (T *)sino_t,
                           p->n, p->nz, p->n_bins, p->d_trig, p->d_angle_order, p->d_partner, p->d_batches, h, inv_ds,
                           (T)p->atten, on);
    else
        hipLaunchKernelGGL((project3d_kernel<T, ZC, NC, false>), grid, dim3(256), 0, s, (const T *)vol_t,
                           (T *)sino_t, p->n, p->nz, p->n_bins, p->d_trig, p->d_angle_order, p->d_partner,
                           p->d_batches, h, inv_ds, (T)p->atten, on);
}

// Sum of the march splits' partial sinograms ([view][bin][z], four slices per element) on
// switched-on workgroups, zero elsewhere (fixed order).
__global__ void k_p3d_reduce(const float4 *__restrict__ part, float4 *__restrict__ out,
                             const uint8_t *__restrict__ wg_on, const int *__restrict__ view_batch, int n_angles, int nb,
                             int nz, int ngroups, int zc, int nzc, int nsplit, long long total4) {
    const int nz4 = nz / 4;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total4; i += (long long)gridDim.x * blockDim.x) {
        const int z = (int)(i % nz4) * 4;
        const long long ab = i / nz4;
        const int bin = (int)(ab % nb), a = (int)(ab / nb);
        const int vb = view_batch[a];
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (vb >= 0) {
            const int b = (vb & 1) ? nb - 1 - bin : bin;
            if (!wg_on || wg_on[((size_t)(vb >> 1) * ngroups + b / kPB) * nzc + z / zc])
                for (int k = 0; k < nsplit; ++k) {
                    const float4 w = part[(size_t)k * total4 + i];
                    v.x += w.x; v.y += w.y; v.z += w.z; v.w += w.w;
                }
        }
        out[i] = v;
    }
}

template <int ZC, int NC, bool PAIR, bool SKIP, int CM, bool LIST, bool QUEUE>
static void fp3d_dma_launch_k(sipo_plan p, const void *vol_t, void *sino_t, hipStream_t s, const uint8_t *on,
                              const SplitSpec &sp, const PrimalFuse &fz, const StepList &sl) {
    const double h = 2.0 / p->n, inv_ds = 0.5 * p->n_bins;
    const int ns = sp.parts > 1 ? sp.parts : 1;
    const dim3 grid((p->n_bins + kPB - 1) / kPB, p->n_batches, ((p->nz + ZC - 1) / ZC) * ns);
    dim3 g = grid;
    if constexpr (QUEUE) {
        // persistent grid: queue_per_cu workgroups per CU (at most as many as fit), at most one per tile
        static int occ[64] = {}, cus[64] = {};
        const int d = p->device >= 0 && p->device < 64 ? p->device : 0;
        if (!occ[d]) {
            int o = 0, c = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, project3d_dma_kernel<ZC, NC, PAIR, SKIP, CM, LIST, true>,
                                                             256, 0) != hipSuccess || o < 1)
                o = 1;
            if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess || c < 1)
                c = 1;
            cus[d] = c;
            occ[d] = o;
        }
        const int per_cu = sl.queue_per_cu > 0 ? std::min(sl.queue_per_cu, occ[d]) : occ[d];
        g = dim3((unsigned)std::max(1, std::min(sl.n_items, per_cu * cus[d])));
    }
    hipLaunchKernelGGL((project3d_dma_kernel<ZC, NC, PAIR, SKIP, CM, LIST, QUEUE>), g, dim3(256), 0, s,
                       (const float *)vol_t, (float *)(ns > 1 ? sp.partial : sino_t), p->n, p->nz, p->n_bins, p->d_trig,
                       p->d_angle_order, p->d_partner, p->d_batches, p->d_ranges, p->d_vial_rows,
                       (const float4 *)p->d_zero, h, inv_ds, (float)p->atten, on, ns, (long long)p->sino_elems(), fz,
                       sl.steps, sl.count, QUEUE ? sl.items : nullptr, sl.n_items, QUEUE ? sl.queue : nullptr,
                       (int)grid.x, (int)(grid.z / ns));
    if (ns > 1) {
        const long long total4 = (long long)p->sino_elems() / 4;
        hipLaunchKernelGGL(k_p3d_reduce, dim3((unsigned)std::min<long long>((total4 + 255) / 256, 16384)), dim3(256), 0,
                           s, (const float4 *)sp.partial, (float4 *)sino_t, on, p->d_view_batch, p->n_angles, p->n_bins,
                           p->nz, (p->n_bins + kPB - 1) / kPB, ZC, (p->nz + ZC - 1) / ZC, ns, total4);
    }
}

// The listed march of an unsplit solve takes the work queue when the caller set one up (and the
// outputs the queue leaves unwritten are not read); everything else runs one workgroup per tile.
static bool list_queued(const SplitSpec &sp, const PrimalFuse &fz, const StepList &sl) {
    return sl.items && sl.queue && sp.parts <= 1 && (fz.y || sl.off_unread);
}

template <int ZC, int NC, bool PAIR, bool SKIP, int CM, bool LIST>
static void fp3d_dma_launch(sipo_plan p, const void *vol_t, void *sino_t, hipStream_t s, const uint8_t *on,
                            const SplitSpec &sp, const PrimalFuse &fz, const StepList &sl) {
    if constexpr (LIST) {
        if (list_queued(sp, fz, sl)) {
            fp3d_dma_launch_k<ZC, NC, PAIR, SKIP, CM, true, true>(p, vol_t, sino_t, s, on, sp, fz, sl);
            return;
        }
    }
    fp3d_dma_launch_k<ZC, NC, PAIR, SKIP, CM, LIST, false>(p, vol_t, sino_t, s, on, sp, fz, sl);
}

template <int ZC, int NC, bool PAIR, bool SKIP>
static void fp3d_dma_go(sipo_plan p, const void *vol_t, void *sino_t, hipStream_t s, const uint8_t *on,
                        const SplitSpec &sp, const PrimalFuse &fz, const StepList &sl) {
    // 64 slices stage one step per chunk only: three two-step buffers would not fit in LDS.  Step
    // lists (masked solves) stage one or two listed steps per chunk (p3d_list_chunk)
    if constexpr (ZC <= 32) {
        if (sl.steps) {
            if constexpr (ZC <= 16) {
                if (p3d_list_chunk(p, sl) == 2) {
                    fp3d_dma_launch<ZC, NC, PAIR, SKIP, 2, true>(p, vol_t, sino_t, s, on, sp, fz, sl);
                    return;
                }
            }
            fp3d_dma_launch<ZC, NC, PAIR, SKIP, 1, true>(p, vol_t, sino_t, s, on, sp, fz, sl);
            return;
        }
    }
    if (ZC > 32 || p->p3d_cm == 1) fp3d_dma_launch<ZC, NC, PAIR, SKIP, 1, false>(p, vol_t, sino_t, s, on, sp, fz, sl);
    else fp3d_dma_launch<ZC, NC, PAIR, SKIP, (ZC > 32 ? 1 : kDmaMaxCM), false>(p, vol_t, sino_t, s, on, sp, fz, sl);
}

template <int ZC, int NC>
static void fp3d_dma_nc(sipo_plan p, const void *vol_t, void *sino_t, hipStream_t s, const uint8_t *on,
                        const SplitSpec &sp, const PrimalFuse &fz, const StepList &sl) {
    if (p->p3d_pair) {
        if (p->p3d_skip) fp3d_dma_go<ZC, NC, true, true>(p, vol_t, sino_t, s, on, sp, fz, sl);
        else fp3d_dma_go<ZC, NC, true, false>(p, vol_t, sino_t, s, on, sp, fz, sl);
    } else {
        if (p->p3d_skip) fp3d_dma_go<ZC, NC, false, true>(p, vol_t, sino_t, s, on, sp, fz, sl);
        else fp3d_dma_go<ZC, NC, false, false>(p, vol_t, sino_t, s, on, sp, fz, sl);
    }
}

template <typename T, int ZC>
static int fp3d_zc(sipo_plan p, const void *vol_t, void *sino_t, hipStream_t s, const uint8_t *on,
                   const SplitSpec &sp, const PrimalFuse *fuse, const StepList &sl) {
    if constexpr (sizeof(T) == 4 && ZC >= 8) {
        if (p->p3d_dma) {
            if (fuse && sp.parts > 1)
                return fail(SIPO_E_UNSUPPORTED, "3D projector: the fused primal step needs an unsplit march");
            const PrimalFuse fz = fuse ? *fuse : PrimalFuse();
            switch (p->p3d_nc) {
                case 3: fp3d_dma_nc<ZC, 3>(p, vol_t, sino_t, s, on, sp, fz, sl); break;
                case 4: fp3d_dma_nc<ZC, 4>(p, vol_t, sino_t, s, on, sp, fz, sl); break;
                case 6: fp3d_dma_nc<ZC, 6>(p, vol_t, sino_t, s, on, sp, fz, sl); break;
                default: return fail(SIPO_E_UNSUPPORTED, "3D projector: unsupported candidate count");
            }
            return SIPO_OK;
        }
    }
    if (sl.steps) return fail(SIPO_E_UNSUPPORTED, "3D projector: step lists need the asynchronous variant");
    if (fuse) return fail(SIPO_E_UNSUPPORTED, "3D projector: the fused primal step needs the asynchronous variant");
    if constexpr (ZC > 32) {
        return fail(SIPO_E_UNSUPPORTED, "3D projector: %d slices per thread need the asynchronous variant", ZC);
    } else {
    switch (p->p3d_nc) {
        case 3: fp3d_nc<T, ZC, 3>(p, vol_t, sino_t, s, on); break;
        case 4: fp3d_nc<T, ZC, 4>(p, vol_t, sino_t, s, on); break;
        case 6: fp3d_nc<T, ZC, 6>(p, vol_t, sino_t, s, on); break;
        default: return fail(SIPO_E_UNSUPPORTED, "3D projector: unsupported candidate count");
    }
    return SIPO_OK;
    }
}

template <typename T>
static int fp3d(sipo_plan p, const void *vol_t, void *sino_t, hipStream_t s, const uint8_t *on,
                const SplitSpec &sp, const PrimalFuse *fuse, const StepList &sl) {
    int rc;
    switch (p->p3d_zc) {
        case 8: rc = fp3d_zc<T, 8>(p, vol_t, sino_t, s, on, sp, fuse, sl); break;
        case 16: rc = fp3d_zc<T, 16>(p, vol_t, sino_t, s, on, sp, fuse, sl); break;
        case 32:
            if constexpr (sizeof(T) == 4) rc = fp3d_zc<T, 32>(p, vol_t, sino_t, s, on, sp, fuse, sl);
            else rc = fail(SIPO_E_UNSUPPORTED, "3D projector: 32 slices per thread in FP64");
            break;
        case 64:
            if constexpr (sizeof(T) == 4) rc = fp3d_zc<T, 64>(p, vol_t, sino_t, s, on, sp, fuse, sl);
            else rc = fail(SIPO_E_UNSUPPORTED, "3D projector: 64 slices per thread in FP64");
            break;
        default: return fail(SIPO_E_UNSUPPORTED, "3D projector: %d slices per thread", p->p3d_zc);
    }
    if (rc) return rc;
    SIPO_LAUNCHED("project3d_kernel");
    return SIPO_OK;
}

int launch_vol_to_t(sipo_plan p, const void *vol, void *vol_t, hipStream_t s, const uint8_t *tile_on) {
    return transpose_any(p, vol, vol_t, 1, p->nz, p->n * p->n, 0, s, tile_on);
}

int launch_sino_to_t(sipo_plan p, const void *sino, void *sino_t, hipStream_t s) {
    return transpose_any(p, sino, sino_t, p->n_angles, p->nz, p->n_bins, 0, s);
}

int launch_sino_from_t(sipo_plan p, const void *sino_t, void *sino, int accumulate, hipStream_t s) {
    return transpose_any(p, sino_t, sino, p->n_angles, p->n_bins, p->nz, accumulate, s);
}

int launch_mask_to_t(sipo_plan p, const uint8_t *mask, uint8_t *mask_t, hipStream_t s) {
    transpose<uint8_t>(mask, mask_t, p->n_angles, p->nz, p->n_bins, 0, s);
    SIPO_LAUNCHED("transpose_kernel<u8>");
    return SIPO_OK;
}

// Single-slice P through an [x][y] copy of the volume in the caller's plan workspace.
static int fp2d_plan(sipo_plan p, const void *vol, void *sino, int accumulate, hipStream_t s) {
    int rc = check_plan_ws(p);
    if (!rc) rc = launch_tr2d(p->dtype, p->d_geo2d, p->d_items_tr2d, p->n_items_tr2d, vol, p->ws_vol_t(), s);
    return rc ? rc : launch_fp2d(p->dtype, p->p3d_nc, p->n, p->d_geo2d, p->d_items_fp2d, p->n_items_fp2d, vol,
                                 p->ws_vol_t(), sino, accumulate, s);
}

// Internal-layout entry points (see sipo_internal.hpp).  Slice and fallback
// plans have no separate internal layout: they run the slice kernels directly.
int launch_backproject_t(sipo_plan p, const void *sino_t, void *vol, int accumulate, hipStream_t s,
                         const uint8_t *tile_on, const SplitSpec &sp) {
    if (p->p2d_ok)
        return launch_bp2d(p->dtype, bp2d_stage_fits(p->n, p->n_bins), p->d_geo2d, p->d_items_bp2d,
                           p->n_items_bp2d, sino_t, vol, accumulate, s);
    if (!p->fast3d())
        return p->dtype == SIPO_F64 ? bp_slices<double>(p, sino_t, vol, accumulate, s)
                                    : bp_slices<float>(p, sino_t, vol, accumulate, s);
    return p->dtype == SIPO_F64 ? bp3d<double>(p, sino_t, vol, accumulate, s, tile_on, sp)
                                : bp3d<float>(p, sino_t, vol, accumulate, s, tile_on, sp);
}

int launch_project_t(sipo_plan p, const void *vol_t, void *sino_t, hipStream_t s, const uint8_t *wg_on,
                     const SplitSpec &sp, const PrimalFuse *fuse, const StepList &sl) {
    if (fuse && (!p->fast3d() || p->dtype != SIPO_F32 || p->p2d_ok))
        return fail(SIPO_E_UNSUPPORTED, "the fused primal step needs an FP32 3D plan");
    if (sl.steps && (!p->fast3d() || p->p2d_ok || !wg_on || !p->p3d_dma || !p->p3d_list_ok || p->p3d_zc > 32))
        return fail(SIPO_E_UNSUPPORTED, "projector step lists need a 3D plan with the asynchronous projector at "
                    "8, 16 or 32 slices per thread, workgroup flags and n <= %d", kMaxListSteps);
    if (p->p2d_ok) return fp2d_plan(p, vol_t, sino_t, 0, s);
    if (!p->fast3d())
        return p->dtype == SIPO_F64 ? fp_slices<double>(p, vol_t, sino_t, 0, s)
                                    : fp_slices<float>(p, vol_t, sino_t, 0, s);
    return p->dtype == SIPO_F64 ? fp3d<double>(p, vol_t, sino_t, s, wg_on, sp, fuse, sl)
                                : fp3d<float>(p, vol_t, sino_t, s, wg_on, sp, fuse, sl);
}

// ------------------------------------------------------- skip flags (LP solves)
// An LP uses P only on its active rays and P^T only where its constrained voxels (band and gel)
// or the blur around them read the result.  The solver therefore runs the 3D operators with one
// flag per workgroup: a projector workgroup is on when one of its rays (or their opposite rays)
// is active, a backprojector tile when it lies within the PSF radius of a labelled voxel.
// Workgroups that are off write zeros.
static int p3d_zchunks(sipo_plan p) { return (p->nz + p->p3d_zc - 1) / p->p3d_zc; }

size_t p3d_flag_count(sipo_plan p, int zc) {
    if (zc <= 0) zc = p->p3d_zc;
    return p->fast3d() ? (size_t)p->n_batches * ((p->n_bins + kPB - 1) / kPB) * ((p->nz + zc - 1) / zc) : 0;
}

size_t bp3d_flag_count(sipo_plan p, int zc) {
    if (!p->fast3d()) return 0;
    if (zc <= 0) zc = p->bp3d_zc;
    return (size_t)((p->n + kBpTX - 1) / kBpTX) * ((p->n + kBpTY - 1) / kBpTY) * ((p->nz + zc - 1) / zc);
}

__global__ void k_flags_clear(uint8_t *f, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        f[i] = 0;
}

// act_t: [view][bin][z]; view_batch[v] = 2 * batch + (v is the opposite view of a walked one)
__global__ void k_p3d_flags(const uint8_t *__restrict__ act_t, uint8_t *__restrict__ flags,
                            const int *__restrict__ view_batch, int n_angles, int nb, int nz, int ngroups, int zc,
                            int nzc) {
    const long long total = (long long)n_angles * nb * nz;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
        if (!act_t[i]) continue;
        const int z = (int)(i % nz);
        const long long ab = i / nz;
        const int bin = (int)(ab % nb), a = (int)(ab / nb);
        const int vb = view_batch[a];
        if (vb < 0) continue;
        const int b = (vb & 1) ? nb - 1 - bin : bin;
        flags[((size_t)(vb >> 1) * ngroups + b / kPB) * nzc + z / zc] = 1;
    }
}

// labels: [z][y][x]; a labelled voxel switches on every tile within (rx, ry, rz) of it
__global__ void k_bp3d_flags(const uint8_t *__restrict__ lab, uint8_t *__restrict__ flags, int n, int nz, int rx,
                             int ry, int rz, int zc, int gx, int gy, int gz) {
    const long long total = (long long)nz * n * n;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
        if (!lab[i]) continue;
        const int x = (int)(i % n), y = (int)((i / n) % n), z = (int)(i / ((long long)n * n));
        const int tx0 = max(x - rx, 0) / kBpTX, tx1 = min(x + rx, n - 1) / kBpTX;
        const int ty0 = max(y - ry, 0) / kBpTY, ty1 = min(y + ry, n - 1) / kBpTY;
        const int tz0 = max(z - rz, 0) / zc, tz1 = min(z + rz, nz - 1) / zc;
        for (int tz = tz0; tz <= tz1 && tz < gz; ++tz)
            for (int ty = ty0; ty <= ty1 && ty < gy; ++ty)
                for (int tx = tx0; tx <= tx1 && tx < gx; ++tx) flags[((size_t)tz * gy + ty) * gx + tx] = 1;
    }
}

// ------------------------------------------------------ step lists (LP solves)
// In an LP solve the projector reads K z, and z vanishes off the labelled voxels, so K z vanishes
// outside the PSF box around them.  A march step whose staged strip holds no voxel of that box in
// the workgroup's slices contributes exactly zero to every ray of the workgroup; the step lists leave
// such steps out.  Built once per solve from the labels: C[zb] marks the columns (x, y) with a
// labelled voxel in a slice within rz of z chunk zb, R[zb] dilates C by (rx, ry) in the plane.

// C[zb][y][x]: a labelled voxel at (x, y) in slices [zb zc - rz, zb zc + zc - 1 + rz]
__global__ void k_reach_z(const uint8_t *__restrict__ lab, uint8_t *__restrict__ C, int n, int nz, int zc, int nzc,
                          int rz) {
    const long long nn = (long long)n * n, total = nn * nzc;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
        const int zb = (int)(i / nn);
        const long long xy = i - zb * nn;
        const int za = max(zb * zc - rz, 0), ze = min(zb * zc + zc - 1 + rz, nz - 1);
        uint8_t on = 0;
        for (int z = za; z <= ze && !on; ++z) on = lab[(size_t)z * nn + xy];
        C[i] = on ? 1 : 0;
    }
}

// R[zb][y][x]: C set within (rx, ry) of (x, y)
__global__ void k_reach_xy(const uint8_t *__restrict__ C, uint8_t *__restrict__ R, int n, int nzc, int rx, int ry) {
    const long long nn = (long long)n * n, total = nn * nzc;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
        const int zb = (int)(i / nn);
        const int y = (int)((i - zb * nn) / n), x = (int)(i % n);
        const uint8_t *c = C + (size_t)zb * nn;
        uint8_t on = 0;
        for (int yy = max(y - ry, 0); yy <= min(y + ry, n - 1) && !on; ++yy)
            for (int xx = max(x - rx, 0); xx <= min(x + rx, n - 1) && !on; ++xx) on = c[(size_t)yy * n + xx];
        R[i] = on ? 1 : 0;
    }
}

// One workgroup per projector workgroup (flag index wg = (batch ngroups + group) nzc + zb): the steps
// m whose staged cross range [j0, j0 + count) holds a voxel of R[zb], compacted in increasing order.
__global__ void __launch_bounds__(256) k_p3d_steps(const int4 *__restrict__ batches, const int2 *__restrict__ ranges,
                                                   const uint8_t *__restrict__ R, const uint8_t *__restrict__ wg_on,
                                                   int *__restrict__ steps, int *__restrict__ count, int n, int ngroups,
                                                   int nzc) {
    __shared__ int wave_cnt[4];
    const int wg = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int zb = wg % nzc, bg = wg / nzc, group = bg % ngroups, batch = bg / ngroups;
    if (!wg_on[wg]) {
        if (tid == 0) count[wg] = 0;
        return;
    }
    const bool xmajor = batches[batch].z != 0;
    const int2 *rg = ranges + ((size_t)batch * ngroups + group) * n;
    const uint8_t *Rz = R + (size_t)zb * n * n;
    int base = 0;
    for (int m0 = 0; m0 < n; m0 += 256) {
        const int m = m0 + tid;
        bool on = false;
        if (m < n) {
            const int2 r = rg[m];
            const int ja = max(r.x, 0), jb = min(r.x + r.y, n);
            for (int j = ja; j < jb && !on; ++j) on = Rz[xmajor ? (size_t)j * n + m : (size_t)m * n + j] != 0;
        }
        const unsigned long long bal = __ballot(on);
        if (lane == 0) wave_cnt[w] = __popcll(bal);
        __syncthreads();
        int off = base;
        for (int q = 0; q < w; ++q) off += wave_cnt[q];
        const int tot = wave_cnt[0] + wave_cnt[1] + wave_cnt[2] + wave_cnt[3];
        if (on) steps[(size_t)wg * n + off + __popcll(bal & ((1ull << lane) - 1ull))] = m;
        base += tot;
        __syncthreads();
    }
    if (tid == 0) count[wg] = base;
}

int p3d_list_chunk(sipo_plan p, const StepList &sl) {
    if (p->p3d_zc > 16) return 1;   // a two-step ring at 32 slices would not fit beside a second workgroup
    if (sl.chunk == 1 || sl.chunk == 2) return sl.chunk;
    // rule: two steps when every switched-on tile can be resident at once with the two-step ring
    // (its LDS bounds the workgroups per CU; the registers allow at least as many at 16 slices)
    static int cus[64] = {};
    const int d = p->device >= 0 && p->device < 64 ? p->device : 0;
    if (!cus[d]) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess || c < 1) c = 1;
        cus[d] = c;
    }
    const long long ring = 3LL * 2 * (p->p3d_zc / 4) * (kPCR + 1) * 16, lds = ring + 8LL * kMaxListSteps + 256;
    const long long per_cu = (160LL * 1024) / lds;
    return sl.n_on > 0 && sl.n_on <= per_cu * cus[d] ? 2 : 1;
}

bool p3d_steps_ok(sipo_plan p) {
    return p->fast3d() && p->p3d_dma && p->p3d_list_ok && p->d_ranges && p->p3d_zc <= 32;
}

size_t p3d_reach_bytes(sipo_plan p, int zc) {
    if (zc <= 0) zc = p->p3d_zc;
    return p->fast3d() ? 2 * (size_t)((p->nz + zc - 1) / zc) * p->n * p->n : 0;
}

int launch_p3d_steps(sipo_plan p, const uint8_t *labels, const uint8_t *wg_on, uint8_t *reach, int *steps, int *count,
                     hipStream_t s) {
    const size_t cnt = p3d_flag_count(p);
    if (!cnt) return SIPO_OK;
    if (!p3d_steps_ok(p)) return fail(SIPO_E_UNSUPPORTED, "projector step lists do not apply to this plan");
    const int zc = p->p3d_zc, nzc = p3d_zchunks(p), ngroups = (p->n_bins + kPB - 1) / kPB;
    if (cnt != (size_t)p->n_batches * ngroups * nzc) return fail(SIPO_E_INVALID, "projector flag count mismatch");
    const int rx = p->has_psf ? p->taps_d.rx : 0, ry = p->has_psf ? p->taps_d.ry : 0, rz = p->has_psf ? p->taps_d.rz : 0;
    uint8_t *C = reach, *R = reach + (size_t)nzc * p->n * p->n;
    const long long total = (long long)nzc * p->n * p->n;
    const unsigned g = (unsigned)std::min<long long>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(k_reach_z, dim3(g), dim3(256), 0, s, labels, C, p->n, p->nz, zc, nzc, rz);
    hipLaunchKernelGGL(k_reach_xy, dim3(g), dim3(256), 0, s, (const uint8_t *)C, R, p->n, nzc, rx, ry);
    hipLaunchKernelGGL(k_p3d_steps, dim3((unsigned)cnt), dim3(256), 0, s, (const int4 *)p->d_batches,
                       (const int2 *)p->d_ranges, (const uint8_t *)R, wg_on, steps, count, p->n, ngroups, nzc);
    SIPO_LAUNCHED("k_p3d_steps");
    return SIPO_OK;
}

int launch_p3d_flags(sipo_plan p, const uint8_t *act_t, uint8_t *flags, hipStream_t s) {
    const size_t cnt = p3d_flag_count(p);
    if (!cnt) return SIPO_OK;
    hipLaunchKernelGGL(k_flags_clear, dim3((unsigned)std::min<size_t>((cnt + 255) / 256, 4096)), dim3(256), 0, s, flags,
                       (long long)cnt);
    const long long total = (long long)p->n_angles * p->n_bins * p->nz;
    hipLaunchKernelGGL(k_p3d_flags, dim3((unsigned)std::min<long long>((total + 255) / 256, 16384)), dim3(256), 0, s,
                       act_t, flags, p->d_view_batch, p->n_angles, p->n_bins, p->nz, (p->n_bins + kPB - 1) / kPB,
                       p->p3d_zc, p3d_zchunks(p));
    SIPO_LAUNCHED("k_p3d_flags");
    return SIPO_OK;
}

int launch_bp3d_flags(sipo_plan p, const uint8_t *labels, uint8_t *flags, hipStream_t s) {
    const size_t cnt = bp3d_flag_count(p);
    if (!cnt) return SIPO_OK;
    hipLaunchKernelGGL(k_flags_clear, dim3((unsigned)std::min<size_t>((cnt + 255) / 256, 4096)), dim3(256), 0, s, flags,
                       (long long)cnt);
    const int rx = p->has_psf ? p->taps_d.rx : 0, ry = p->has_psf ? p->taps_d.ry : 0, rz = p->has_psf ? p->taps_d.rz : 0;
    const int gx = (p->n + kBpTX - 1) / kBpTX, gy = (p->n + kBpTY - 1) / kBpTY, gz = (p->nz + p->bp3d_zc - 1) / p->bp3d_zc;
    const long long total = (long long)p->nz * p->n * p->n;
    hipLaunchKernelGGL(k_bp3d_flags, dim3((unsigned)std::min<long long>((total + 255) / 256, 16384)), dim3(256), 0, s,
                       labels, flags, p->n, p->nz, rx, ry, rz, p->bp3d_zc, gx, gy, gz);
    SIPO_LAUNCHED("k_bp3d_flags");
    return SIPO_OK;
}

size_t bp3d_need_bytes(sipo_plan p, int zc) {
    if (zc <= 0) zc = p->bp3d_zc;
    return p->fast3d() ? (size_t)((p->nz + zc - 1) / zc) * p->n * p->n : 0;
}

int launch_bp3d_need(sipo_plan p, const uint8_t *labels, uint8_t *scratch, uint8_t *need, hipStream_t s) {
    if (!p->fast3d()) return SIPO_OK;
    const int zc = p->bp3d_zc, nzc = (p->nz + zc - 1) / zc;
    const int rx = p->has_psf ? p->taps_d.rx : 0, ry = p->has_psf ? p->taps_d.ry : 0, rz = p->has_psf ? p->taps_d.rz : 0;
    const long long total = (long long)nzc * p->n * p->n;
    const unsigned g = (unsigned)std::min<long long>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(k_reach_z, dim3(g), dim3(256), 0, s, labels, scratch, p->n, p->nz, zc, nzc, rz);
    hipLaunchKernelGGL(k_reach_xy, dim3(g), dim3(256), 0, s, (const uint8_t *)scratch, need, p->n, nzc, rx, ry);
    SIPO_LAUNCHED("k_reach_xy");
    return SIPO_OK;
}

// ABI-layout entry points: the volume kernels run on z-contiguous copies made in the caller's
// plan workspace.
int launch_backproject(sipo_plan p, const void *sino, void *vol, int accumulate, hipStream_t s) {
    if (!p->fast3d()) return launch_backproject_t(p, sino, vol, accumulate, s);
    int rc = check_plan_ws(p);
    if (!rc) rc = launch_sino_to_t(p, sino, p->ws_sino_t(), s);
    return rc ? rc : launch_backproject_t(p, p->ws_sino_t(), vol, accumulate, s);
}

int launch_project(sipo_plan p, const void *vol, void *sino, int accumulate, hipStream_t s) {
    if (p->p2d_ok) return fp2d_plan(p, vol, sino, accumulate, s);
    if (!p->fast3d())
        return p->dtype == SIPO_F64 ? fp_slices<double>(p, vol, sino, accumulate, s)
                                    : fp_slices<float>(p, vol, sino, accumulate, s);
    int rc = check_plan_ws(p);
    if (!rc) rc = launch_vol_to_t(p, vol, p->ws_vol_t(), s);
    if (!rc) rc = launch_project_t(p, p->ws_vol_t(), p->ws_sino_t(), s);
    return rc ? rc : launch_sino_from_t(p, p->ws_sino_t(), sino, accumulate, s);
}

}  // namespace sipo
