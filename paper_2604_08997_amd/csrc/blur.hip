// Object-space PSF K (Eq. 1-3): separable convolution with zero boundary,
// fused into one pass over HBM.
//
// A workgroup owns a 64 x 16 (x, y) tile and a chunk of slices.  It streams
// the slices in z order: each slice tile (with its x/y halo) is staged in LDS,
// blurred along x and then y, and the xy-blurred values of a thread's four
// rows are pushed through a register ring of 2 rz + 1 slices; once the ring
// is full the z taps produce one output slice.  The next slice is fetched into
// registers while the current one is being blurred, so the HBM stream does not
// wait on the two LDS passes.  Every input slice is read once per tile (plus
// halos, mostly from L2) and every output written once.
//
// The x and y radii share one compile-time radius RXY = max(rx, ry); an axis
// with a smaller radius gets its taps zero-padded to that width.
#include "sipo_internal.hpp"

namespace sipo {

constexpr int kBTX = 64, kBTY = 16, kBRows = kBTY / 4;   // tile; 256 threads = 64 x 4, 4 rows per thread
constexpr int kBlurMaskedPF = 2;   // slices fetched ahead by tile-masked launches

// PF is the number of slices fetched ahead.  PF = 1 (full volumes, many workgroups per CU): guarded
// loads, one slice ahead.  PF > 1 (tile-masked launches, few workgroups whose serial slice walk is the
// whole cost): every load is unconditional, from an address clamped into the volume, with the values
// outside it selected to zero, so the compiler can count them in its memory waits; slices are fetched PF
// ahead into statically indexed register slots, and the walk is padded to a multiple of PF (a padded slice
// re-reads the last walked one and stores nothing).
// TOUT (FP32, tile-masked, z chunks and nz multiples of 4): the output goes to the projector's
// z-contiguous layout [y][x][z] instead of [z][y][x]: a thread keeps its rows' last four output slices
// and stores them as one 16-byte word, so no separate transpose follows; switched-off tiles write
// nothing (that layout holds zeros there).
template <typename T, int RXY, int RZ, int PF, bool TOUT = false>
__global__ void __launch_bounds__(256) blur_kernel(const T *__restrict__ in, T *__restrict__ out, int n, int nz,
                                                   Taps<T> tp, int zchunk, const uint8_t *__restrict__ tile_on,
                                                   int zero_off) {
    static_assert(!TOUT || (sizeof(T) == 4 && PF > 1), "z-contiguous output: FP32 tile-masked launches");
    constexpr int RW = kBTX + 2 * RXY, RH = kBTY + 2 * RXY;
    constexpr int LR = (RH + 3) / 4;   // staged rows per thread
    __shared__ T raw[RH][RW + 1];
    __shared__ T xb[RH][kBTX + 1];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int3 tile = xcd_tile<0>();   // x rotated per z chunk: row neighbours share halos in L2
    const int x0 = tile.x * kBTX, y0 = tile.y * kBTY;
    const int z0 = tile.z * zchunk;
    const int zend = min(nz, z0 + zchunk);
    const size_t plane = (size_t)n * n;
    if (tile_on && !tile_on[((size_t)tile.z * gridDim.y + tile.y) * gridDim.x + tile.x]) {
        if (zero_off) {
            const int gx = x0 + tx;
            for (int zo = z0; zo < zend; ++zo)
#pragma unroll
                for (int j = 0; j < kBRows; ++j) {
                    const int gy = y0 + ty + 4 * j;
                    if (gx < n && gy < n) out[(size_t)zo * plane + (size_t)gy * n + gx] = (T)0;
                }
        }
        return;
    }
    const int gxm = x0 - RXY + tx, gxh = x0 - RXY + kBTX + tx;
    const bool okm = gxm >= 0 && gxm < n, okh = tx < 2 * RXY && gxh >= 0 && gxh < n;
    const int zfirst = z0 - RZ, zlast = zend + RZ;   // walked input slices [zfirst, zlast)

    T pm[PF][LR], ph[PF][LR];
    // PF = 1: values outside the volume are zeroed as they are loaded.  PF > 1: the slots hold the raw loads
    // and stage() zeroes them, so no wait is needed until a slot is staged.
    auto fetch = [&](T (&m)[LR], T (&hh)[LR], int zi) {
        if constexpr (PF == 1) {
            const bool zok = zi >= 0 && zi < nz;
            const T *src = in + (size_t)(zok ? zi : 0) * plane;
#pragma unroll
            for (int k = 0; k < LR; ++k) {
                const int ly = ty + 4 * k, gy = y0 - RXY + ly;
                const bool yok = zok && ly < RH && gy >= 0 && gy < n;
                m[k] = (yok && okm) ? src[(size_t)gy * n + gxm] : (T)0;
                hh[k] = (yok && okh) ? src[(size_t)gy * n + gxh] : (T)0;
            }
        } else {
            const int za = min(max(min(zi, zlast - 1), 0), nz - 1);
            const T *src = in + (size_t)za * plane;
            const int xm = min(max(gxm, 0), n - 1), xh = min(max(gxh, 0), n - 1);
#pragma unroll
            for (int k = 0; k < LR; ++k) {
                const size_t row = (size_t)min(max(y0 - RXY + ty + 4 * k, 0), n - 1) * n;
                m[k] = src[row + xm];
                hh[k] = src[row + xh];
            }
        }
    };
    auto stage = [&](const T (&m)[LR], const T (&hh)[LR], int zi) {
        const bool zok = PF == 1 || (zi >= 0 && zi < nz && zi < zlast);
#pragma unroll
        for (int k = 0; k < LR; ++k) {
            const int ly = ty + 4 * k, gy = y0 - RXY + ly;
            const bool yok = PF == 1 || (zok && gy >= 0 && gy < n);
            if (ly < RH) {
                raw[ly][tx] = (PF == 1 || (yok && okm)) ? m[k] : (T)0;
                if (tx < 2 * RXY) raw[ly][kBTX + tx] = (PF == 1 || (yok && okh)) ? hh[k] : (T)0;
            }
        }
    };

    T ring[kBRows][2 * RZ + 1];
#pragma unroll
    for (int j = 0; j < kBRows; ++j)
#pragma unroll
        for (int m = 0; m < 2 * RZ + 1; ++m) ring[j][m] = (T)0;
    T zq[TOUT ? kBRows : 1][4];   // TOUT: the last four output slices of each row

    // x and y passes of the staged slice zi, the z ring, and output slice zi - RZ
    auto blur_slice = [&](int zi) {
#pragma unroll
        for (int k = 0; k < LR; ++k) {
            const int ly = ty + 4 * k;
            if (ly < RH) {
                T s = (T)0;
#pragma unroll
                for (int d = 0; d <= 2 * RXY; ++d) s = fma(tp.kx[d], raw[ly][tx + d], s);
                xb[ly][tx] = s;
            }
        }
        __syncthreads();
        T v[kBRows];
#pragma unroll
        for (int j = 0; j < kBRows; ++j) {
            T s = (T)0;
#pragma unroll
            for (int d = 0; d <= 2 * RXY; ++d) s = fma(tp.ky[d], xb[ty + 4 * j + d][tx], s);
            v[j] = s;
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
                if constexpr (TOUT) {
                    zq[j][0] = zq[j][1];
                    zq[j][1] = zq[j][2];
                    zq[j][2] = zq[j][3];
                    zq[j][3] = s;
                    if (((zo - z0) & 3) == 3 && gx < n && gy < n)
                        *(float4 *)(out + ((size_t)gy * n + gx) * nz + (zo - 3)) =
                            make_float4(zq[j][0], zq[j][1], zq[j][2], zq[j][3]);
                } else {
                    if (gx < n && gy < n) out[(size_t)zo * plane + (size_t)gy * n + gx] = s;
                }
            }
        }
    };

    if constexpr (PF == 1) {
        fetch(pm[0], ph[0], zfirst);
        for (int zi = zfirst; zi < zlast; ++zi) {
            stage(pm[0], ph[0], zi);
            __syncthreads();
            if (zi + 1 < zlast) fetch(pm[0], ph[0], zi + 1);
            blur_slice(zi);
        }
    } else {
        const int zpad = zfirst + (zlast - zfirst + PF - 1) / PF * PF;
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            fetch(pm[q], ph[q], zfirst + q);
            asm volatile("" ::: "memory");   // slot q's loads issue before slot q + 1's (the waits count in order)
        }
        for (int zb = zfirst; zb < zpad; zb += PF) {
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                stage(pm[q], ph[q], zb + q);
                __syncthreads();
                fetch(pm[q], ph[q], zb + q + PF);
                blur_slice(zb + q);
            }
        }
    }
}

// Re-centre an axis' taps of radius r on radius R >= r (zeros outside).
template <typename T>
static void pad_taps(T *k, int r, int R) {
    T tmp[2 * kMaxR + 1];
    for (int d = 0; d <= 2 * R; ++d) {
        const int o = d - R + r;
        tmp[d] = (o >= 0 && o <= 2 * r) ? k[o] : (T)0;
    }
    for (int d = 0; d <= 2 * kMaxR; ++d) k[d] = d <= 2 * R ? tmp[d] : (T)0;
}

// z chunk: enough workgroups to fill the chip (about eight per CU) without
// letting the z halo dominate.
static int pick_zchunk(int n, int nz, int rz) {
    const long tiles = (long)((n + kBTX - 1) / kBTX) * ((n + kBTY - 1) / kBTY);
    long zc = (tiles * nz + 2047) / 2048;
    zc = std::max<long>(zc, std::max(8, 2 * rz));
    return (int)std::min<long>(zc, nz);
}

static int blur_zchunk(sipo_plan p) {
    const int rz = p->dtype == SIPO_F64 ? p->taps_d.rz : p->taps_f.rz;
    return p->blur_zc > 0 ? std::min(p->blur_zc, p->nz) : pick_zchunk(p->n, p->nz, rz);
}

size_t blur_tile_count(sipo_plan p, int zc) {
    if (!p->has_psf) return 0;
    zc = zc > 0 ? std::min(zc, p->nz) : blur_zchunk(p);
    return (size_t)((p->n + kBTX - 1) / kBTX) * ((p->n + kBTY - 1) / kBTY) * ((p->nz + zc - 1) / zc);
}

// own[tile of a labelled voxel] = 1; reach[every tile within (rx, ry, rz) of it] = 1
__global__ void k_blur_flags(const uint8_t *__restrict__ lab, uint8_t *__restrict__ own, uint8_t *__restrict__ reach,
                             int n, int nz, int rx, int ry, int rz, int zc, int gx, int gy, int gz) {
    const long long total = (long long)nz * n * n;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
        if (!lab[i]) continue;
        const int x = (int)(i % n), y = (int)((i / n) % n), z = (int)(i / ((long long)n * n));
        own[((size_t)(z / zc) * gy + y / kBTY) * gx + x / kBTX] = 1;
        const int tx0 = max(x - rx, 0) / kBTX, tx1 = min(x + rx, n - 1) / kBTX;
        const int ty0 = max(y - ry, 0) / kBTY, ty1 = min(y + ry, n - 1) / kBTY;
        const int tz0 = max(z - rz, 0) / zc, tz1 = min(z + rz, nz - 1) / zc;
        for (int tz = tz0; tz <= tz1 && tz < gz; ++tz)
            for (int ty = ty0; ty <= ty1 && ty < gy; ++ty)
                for (int tx = tx0; tx <= tx1 && tx < gx; ++tx) reach[((size_t)tz * gy + ty) * gx + tx] = 1;
    }
}

__global__ void k_blur_flags_clear(uint8_t *a, uint8_t *b, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        a[i] = b[i] = 0;
}

int launch_blur_flags(sipo_plan p, const uint8_t *labels, uint8_t *own, uint8_t *reach, hipStream_t s) {
    const size_t cnt = blur_tile_count(p);
    if (!cnt) return SIPO_OK;
    const int zc = blur_zchunk(p);
    const int gx = (p->n + kBTX - 1) / kBTX, gy = (p->n + kBTY - 1) / kBTY, gz = (p->nz + zc - 1) / zc;
    hipLaunchKernelGGL(k_blur_flags_clear, dim3((unsigned)std::min<size_t>((cnt + 255) / 256, 4096)), dim3(256), 0, s,
                       own, reach, (long long)cnt);
    const int rx = p->taps_d.rx, ry = p->taps_d.ry, rz = p->taps_d.rz;
    const long long total = (long long)p->nz * p->n * p->n;
    hipLaunchKernelGGL(k_blur_flags, dim3((unsigned)std::min<long long>((total + 255) / 256, 16384)), dim3(256), 0, s,
                       labels, own, reach, p->n, p->nz, rx, ry, rz, zc, gx, gy, gz);
    SIPO_LAUNCHED("k_blur_flags");
    return SIPO_OK;
}

size_t vol_t_tile_count(sipo_plan p) {
    return (size_t)(((long long)p->n * p->n + kTrCols - 1) / kTrCols) * ((p->nz + kTrRows - 1) / kTrRows);
}

// tflags[t] = 1 when transpose tile t (kTrRows slices x kTrCols consecutive (y n + x)
// columns) holds a voxel of a blur tile that is on in `reach`
__global__ void k_vol_t_flags(const uint8_t *__restrict__ reach, uint8_t *__restrict__ tflags, int n, int nz, int zc,
                              int gx, int gy, int tcols, int trows) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= tcols * trows) return;
    const int cb = t % tcols, rb = t / tcols;
    const long long c0 = (long long)kTrCols * cb, c1 = min(c0 + kTrCols - 1, (long long)n * n - 1);
    const int z0 = kTrRows * rb, z1 = min(z0 + kTrRows - 1, nz - 1);
    uint8_t on = 0;
    for (int y = (int)(c0 / n); y <= (int)(c1 / n) && !on; ++y) {
        const int xa = (int)max(c0 - (long long)y * n, 0LL), xb = (int)min(c1 - (long long)y * n, (long long)n - 1);
        for (int bz = z0 / zc; bz <= z1 / zc && !on; ++bz)
            for (int bx = xa / kBTX; bx <= xb / kBTX && !on; ++bx) on = reach[((size_t)bz * gy + y / kBTY) * gx + bx];
    }
    tflags[t] = on ? 1 : 0;
}

int launch_vol_t_flags(sipo_plan p, const uint8_t *reach, uint8_t *tflags, hipStream_t s) {
    if (!blur_tile_count(p)) return SIPO_OK;
    const int zc = blur_zchunk(p);
    const int gx = (p->n + kBTX - 1) / kBTX, gy = (p->n + kBTY - 1) / kBTY;
    const int tcols = (int)(((long long)p->n * p->n + kTrCols - 1) / kTrCols);
    const int trows = (p->nz + kTrRows - 1) / kTrRows;
    hipLaunchKernelGGL(k_vol_t_flags, dim3((tcols * trows + 255) / 256), dim3(256), 0, s, reach, tflags, p->n, p->nz, zc,
                       gx, gy, tcols, trows);
    SIPO_LAUNCHED("k_vol_t_flags");
    return SIPO_OK;
}

template <typename T, int RXY, int RZ>
static void launch_r(const Taps<T> &tp, const void *in, void *out, int n, int nz, int zchunk, hipStream_t s,
                     const uint8_t *on, int zero_off, bool tout) {
    const dim3 grid((n + kBTX - 1) / kBTX, (n + kBTY - 1) / kBTY, (nz + zchunk - 1) / zchunk);
    if constexpr (sizeof(T) == 4) {
        if (tout) {
            hipLaunchKernelGGL((blur_kernel<T, RXY, RZ, kBlurMaskedPF, true>), grid, dim3(kBTX, 4), 0, s, (const T *)in,
                               (T *)out, n, nz, tp, zchunk, on, 0);
            return;
        }
    }
    if (on)
        hipLaunchKernelGGL((blur_kernel<T, RXY, RZ, kBlurMaskedPF>), grid, dim3(kBTX, 4), 0, s, (const T *)in,
                           (T *)out, n, nz, tp, zchunk, on, zero_off);
    else
        hipLaunchKernelGGL((blur_kernel<T, RXY, RZ, 1>), grid, dim3(kBTX, 4), 0, s, (const T *)in, (T *)out, n, nz,
                           tp, zchunk, on, zero_off);
}

template <typename T, int RXY>
static int launch_rz(const Taps<T> &tp, const void *in, void *out, int n, int nz, int zc, hipStream_t s,
                     const uint8_t *on, int zero_off, bool tout) {
    switch (tp.rz) {
        case 0: launch_r<T, RXY, 0>(tp, in, out, n, nz, zc, s, on, zero_off, tout); break;
        case 1: launch_r<T, RXY, 1>(tp, in, out, n, nz, zc, s, on, zero_off, tout); break;
        case 2: launch_r<T, RXY, 2>(tp, in, out, n, nz, zc, s, on, zero_off, tout); break;
        case 3: launch_r<T, RXY, 3>(tp, in, out, n, nz, zc, s, on, zero_off, tout); break;
        case 4: launch_r<T, RXY, 4>(tp, in, out, n, nz, zc, s, on, zero_off, tout); break;
        case 5: launch_r<T, RXY, 5>(tp, in, out, n, nz, zc, s, on, zero_off, tout); break;
        case 6: launch_r<T, RXY, 6>(tp, in, out, n, nz, zc, s, on, zero_off, tout); break;
        case 7: launch_r<T, RXY, 7>(tp, in, out, n, nz, zc, s, on, zero_off, tout); break;
        case 8: launch_r<T, RXY, 8>(tp, in, out, n, nz, zc, s, on, zero_off, tout); break;
        default: return fail(SIPO_E_UNSUPPORTED, "PSF z radius %d > %d", tp.rz, kMaxR);
    }
    return SIPO_OK;
}

template <typename T>
static int blur_dispatch(sipo_plan p, const Taps<T> &taps, const void *in, void *out, hipStream_t s,
                         const uint8_t *on, int zero_off, bool tout = false) {
    Taps<T> tp = taps;
    const int R = std::max(tp.rx, tp.ry);
    pad_taps(tp.kx, tp.rx, R);
    pad_taps(tp.ky, tp.ry, R);
    tp.rx = tp.ry = R;
    const int zc = blur_zchunk(p);
    int rc;
    switch (R) {
        case 0: rc = launch_rz<T, 0>(tp, in, out, p->n, p->nz, zc, s, on, zero_off, tout); break;
        case 1: rc = launch_rz<T, 1>(tp, in, out, p->n, p->nz, zc, s, on, zero_off, tout); break;
        case 2: rc = launch_rz<T, 2>(tp, in, out, p->n, p->nz, zc, s, on, zero_off, tout); break;
        case 3: rc = launch_rz<T, 3>(tp, in, out, p->n, p->nz, zc, s, on, zero_off, tout); break;
        case 4: rc = launch_rz<T, 4>(tp, in, out, p->n, p->nz, zc, s, on, zero_off, tout); break;
        case 5: rc = launch_rz<T, 5>(tp, in, out, p->n, p->nz, zc, s, on, zero_off, tout); break;
        case 6: rc = launch_rz<T, 6>(tp, in, out, p->n, p->nz, zc, s, on, zero_off, tout); break;
        case 7: rc = launch_rz<T, 7>(tp, in, out, p->n, p->nz, zc, s, on, zero_off, tout); break;
        case 8: rc = launch_rz<T, 8>(tp, in, out, p->n, p->nz, zc, s, on, zero_off, tout); break;
        default: return fail(SIPO_E_UNSUPPORTED, "PSF xy radius %d > %d", R, kMaxR);
    }
    if (rc) return rc;
    SIPO_LAUNCHED("blur_kernel");
    return SIPO_OK;
}

int launch_blur(sipo_plan p, const void *in, void *out, hipStream_t s, const uint8_t *tile_on, int zero_off) {
    if (!p->has_psf) {
        SIPO_HIP(hipMemcpyAsync(out, in, p->vol_elems() * p->elem_bytes(), hipMemcpyDeviceToDevice, s));
        return SIPO_OK;
    }
    return p->dtype == SIPO_F64 ? blur_dispatch<double>(p, p->taps_d, in, out, s, tile_on, zero_off)
                                : blur_dispatch<float>(p, p->taps_f, in, out, s, tile_on, zero_off);
}

bool blur_to_t_ok(sipo_plan p) {
    return p->has_psf && p->dtype == SIPO_F32 && p->fast3d() && p->nz % 4 == 0 && blur_zchunk(p) % 4 == 0;
}

int launch_blur_to_t(sipo_plan p, const void *in, void *vol_t, hipStream_t s, const uint8_t *tile_on) {
    if (!blur_to_t_ok(p) || !tile_on)
        return fail(SIPO_E_UNSUPPORTED, "blur into the projector's layout: FP32 tile-masked 3D launches with z chunks "
                                        "and slice counts multiple of 4");
    return blur_dispatch<float>(p, p->taps_f, in, vol_t, s, tile_on, 0, true);
}

}  // namespace sipo
