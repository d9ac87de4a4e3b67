// Internal declarations shared by the SiPO HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <vector>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>

#include "sipo.h"

namespace sipo {

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...);
int fail(int code, const char *fmt, ...);

#define SIPO_HIP(call)                                                                  \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return ::sipo::fail(SIPO_E_DEVICE, "%s failed: %s (%s:%d)", #call,          \
                                hipGetErrorString(e_), __FILE__, __LINE__);             \
    } while (0)

#define SIPO_LAUNCHED(name)                                                             \
    do {                                                                                \
        hipError_t e_ = hipGetLastError();                                              \
        if (e_ != hipSuccess)                                                           \
            return ::sipo::fail(SIPO_E_DEVICE, "launch of %s failed: %s", name,         \
                                hipGetErrorString(e_));                                 \
    } while (0)

#define SIPO_TRY(call)                                                                  \
    do {                                                                                \
        int rc_ = (call);                                                               \
        if (rc_ != SIPO_OK) return rc_;                                                 \
    } while (0)

#define SIPO_REQUIRE(cond, ...)                                                         \
    do {                                                                                \
        if (!(cond)) return ::sipo::fail(SIPO_E_INVALID, __VA_ARGS__);                  \
    } while (0)

// --------------------------------------------------------------- PSF taps
// Taps travel to kernels by value (kernel argument space), in both precisions.
constexpr int kMaxR = 8;
template <typename T>
struct Taps {
    int rx, ry, rz;
    T kx[2 * kMaxR + 1], ky[2 * kMaxR + 1], kz[2 * kMaxR + 1];
};

// -------------------------------------------------------------------- plan
// The plan's operator workspace is caller memory (sipo_plan_set_workspace).  It holds, in order:
// a reduction area (per-workgroup partials of the metric passes, the maximum of the active-ray
// test), the z-contiguous copy of a volume (fast 3D plans: [y][x][z] input of the projector;
// single-slice plans: the [x][y] copy read by rays that march along x) and the z-contiguous
// sinogram ([view][bin][z], fast 3D plans).  Each part starts on a 256-byte boundary.
constexpr size_t kPlanRedBytes = 1 << 17;
inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Geo2D;

}  // namespace sipo

struct sipo_plan_s {
    int n, nz, n_angles, n_bins;
    double atten;
    sipo_dtype dtype;
    int device;
    bool has_psf;
    sipo::Taps<float> taps_f;
    sipo::Taps<double> taps_d;
    double2 *d_trig;        // [n_angles] (sin, cos)
    size_t table_bytes;     // device bytes of the plan's own tables (everything allocated below)
    void *ws;               // caller workspace for the standalone operator calls (not owned), or NULL
    size_t ws_bytes;
    // per-angle march axis split, on the host, for launch decisions
    int n_xmajor;
    int *d_angle_order;     // views the 3D projector walks: x-major first, then y-major
                            // (only the first view of each opposite pair when p3d_pair)
    int *d_partner;         // [n_angles]: index of the opposite view (theta + pi), or -1
    int *d_view_batch;      // [n_angles]: 2 * projector batch (+1 for the opposite view of a walked one), or -1
    // view batches of the 3D projector: (first index into d_angle_order, count, x-major flag, unused)
    int n_batches;
    int4 *d_batches;
    bool p3d_ok;            // every batch fits the projector's LDS strip
    bool p3d_pair;          // every view has an opposite view: the projector walks pairs
    int p3d_nc;             // candidate voxels per ray step of the 3D projector (0 = unsupported)
    int p3d_zc;             // slices per projector thread (set by defaults or sipo_plan_autotune)
    bool p3d_dma_ok;        // the asynchronous-staging projector applies (FP32, nz % 4 == 0, ranges fit)
    bool p3d_list_ok;       // its step-list variant applies (n and every staged range fit the packed records)
    bool p3d_dma;           // use it (default when it applies; sipo_plan_autotune may switch)
    bool p3d_skip;          // asynchronous projector: lanes skip candidates outside their ray's reach
    int p3d_cm;             // asynchronous projector: march steps per staged chunk (1 or 2)
    int2 *d_ranges;         // [n_batches][bin groups][steps]: staged cross range (j0, count)
    int2 *d_vial_rows;      // [n]: first and last index along a grid line inside the vial
    void *d_zero;           // 256 zero bytes (source of empty staging slots)
    int n_walk;             // views the projector walks (entries of d_angle_order)
    bool p2d_ok;            // single-slice plan served by the 2D kernels
    sipo::Geo2D *d_geo2d;   // this plan as a one-instance batch
    int4 *d_items_bp2d, *d_items_fp2d, *d_items_tr2d;
    int n_items_bp2d, n_items_fp2d, n_items_tr2d;
    int blur_zc;            // slices per blur workgroup (0 = built-in choice)
    int bp3d_zc;            // slices per 3D backprojector thread (8 or 16 in FP64; 8, 16 or 32 in FP32)
    bool bp3d_ok;           // the 3D backprojector's bin window fits its LDS tile
    bool fast3d() const { return nz > 1 && p3d_ok && bp3d_ok; }
    size_t vol_elems() const { return (size_t)nz * n * n; }
    size_t sino_elems() const { return (size_t)n_angles * nz * n_bins; }
    size_t elem_bytes() const { return dtype == SIPO_F64 ? 8 : 4; }
    // workspace layout (see kPlanRedBytes)
    size_t ws_vol_t_bytes() const { return (p2d_ok || fast3d()) ? sipo::align256(vol_elems() * elem_bytes()) : 0; }
    size_t ws_sino_t_bytes() const { return fast3d() ? sipo::align256(sino_elems() * elem_bytes()) : 0; }
    size_t ws_need() const { return sipo::kPlanRedBytes + ws_vol_t_bytes() + ws_sino_t_bytes(); }
    void *ws_red() const { return ws; }
    void *ws_vol_t() const { return (char *)ws + sipo::kPlanRedBytes; }
    void *ws_sino_t() const { return (char *)ws + sipo::kPlanRedBytes + ws_vol_t_bytes(); }
};

namespace sipo {

int check_plan(sipo_plan p);
// SIPO_E_WORKSPACE unless the caller has attached a large enough workspace to the plan
int check_plan_ws(sipo_plan p);
// hipMalloc of a plan table, counted in p->table_bytes
int plan_alloc(sipo_plan p, void **ptr, size_t bytes);

// Tile coordinates (x, y, z) of this workgroup, spread over the XCDs.  Workgroups reach the eight
// XCDs in turn by linear id, so with x taken straight from blockIdx a grid whose x extent is a
// multiple of eight would pin each x column of tiles to one XCD; a masked launch, whose live tiles
// cluster in a few columns, would then run on a few XCDs.  x is rotated by the index of the run of
// RY consecutive y tiles (RY = 0: the whole y extent, i.e. by z alone), so every XCD gets every
// column while a run of RY y-neighbours stays on one XCD and shares its L2.  A bijection of the grid.
template <int RY>
__device__ __forceinline__ int3 xcd_tile() {
    const unsigned ry = RY > 0 ? RY : gridDim.y;
    const unsigned q = blockIdx.y / ry + ((gridDim.y + ry - 1) / ry) * blockIdx.z;
    return make_int3((int)((blockIdx.x + q) % gridDim.x), (int)blockIdx.y, (int)blockIdx.z);
}

// Launchers (return sipo_status).
int launch_backproject(sipo_plan p, const void *sino, void *vol, int accumulate, hipStream_t s);
int launch_project(sipo_plan p, const void *vol, void *sino, int accumulate, hipStream_t s);
// tile_on: optional flags per blur tile (see blur_tile_count); a tile that is off is skipped, or,
// with zero_off, has its output set to zero without reading the input.
int launch_blur(sipo_plan p, const void *in, void *out, hipStream_t s, const uint8_t *tile_on = nullptr,
                int zero_off = 0);
// K of a z that vanishes off the switched-on tiles' reach, written straight into the projector's
// z-contiguous layout (the input of launch_project_t) for the tiles on in tile_on; the layout must
// hold zeros elsewhere.  FP32 3D plans whose blur z chunk and slice count are multiples of 4.
bool blur_to_t_ok(sipo_plan p);
int launch_blur_to_t(sipo_plan p, const void *in, void *vol_t, hipStream_t s, const uint8_t *tile_on);
// Blur tiles of the plan's current tuning (0 without a PSF), and their flags from a label volume
// [z][y][x]: own = the tile holds a labelled voxel, reach = a labelled voxel lies within the PSF
// radius of the tile (elsewhere the blur of a field supported on labelled voxels is zero).
size_t blur_tile_count(sipo_plan p, int zc = 0);   // zc > 0: at zc slices per tile
int launch_blur_flags(sipo_plan p, const uint8_t *labels, uint8_t *own, uint8_t *reach, hipStream_t s);
// Internal 3D layouts (fast3d plans): sinograms [view][bin][z] ("sino_t") and, as
// the projector's input, volumes [y][x][z] ("vol_t"); both keep z contiguous.
// Volumes produced by the backprojector stay in the ABI layout [z][y][x].
// tile_on / wg_on: optional per-workgroup flags of an LP solve (nullptr = the full operator);
// workgroups that are off write zeros.  SplitSpec: the 3D kernels' serial walk (march steps of
// the asynchronous projector, views of the backprojector) split over `parts` workgroups whose
// partial sums go to `partial` (parts x the output's elements) and are then added in a fixed
// order; parts <= 1 = no split.  keep_off: the fixed-order sum leaves the output of switched-off
// tiles as it is instead of writing zeros (for outputs that are only read near switched-on tiles).
struct SplitSpec {
    int parts = 1;
    void *partial = nullptr;
    bool keep_off = false;
    // masked backprojector: per z chunk of its slices, row and column, whether any voxel of the
    // column in the chunk lies within the PSF box of a labelled voxel (launch_bp3d_need); voxels
    // of the other columns are stored as zero
    const uint8_t *need = nullptr;
};
int launch_backproject_t(sipo_plan p, const void *sino_t, void *vol, int accumulate, hipStream_t s,
                         const uint8_t *tile_on = nullptr, const SplitSpec &sp = SplitSpec());
// Primal step of an LP solve fused into the asynchronous projector's output (FP32, no splits):
// instead of storing q = P x, a ray's lane applies t.y = max(0, y - tau_fac T_j q) and
// y <- w ((1 + rho) t.y - rho y) + (1 - w) y0 on its active elements and stores y and t.y; q is
// not stored, and workgroups that are off store nothing.  Arrays are the instance's fields in the
// projector's output layout; the scalars are read from device memory when the kernel runs.
struct PrimalFuse {
    float *y = nullptr, *yt = nullptr;
    const float *Tj = nullptr, *y0 = nullptr;
    const uint8_t *act = nullptr;
    const double *tau_fac = nullptr, *w_rho = nullptr;   // w_rho[0] = w, w_rho[1] = rho
};
// March-step lists of the asynchronous projector in an LP solve: per projector workgroup (the
// index of its skip flag), `count` steps listed in `steps` (n entries reserved per workgroup), in
// increasing order; the workgroup walks those steps only.  nullptr = every step.
struct StepList {
    const int *steps = nullptr;
    const int *count = nullptr;
    // optional work queue (unsplit march only): the switched-on workgroups' flag indices, longest
    // list first, and two zeroed int counters that the projector leaves zeroed
    const int *items = nullptr;
    int n_items = 0;
    int *queue = nullptr;
    int queue_per_cu = 0;   // persistent workgroups per CU (0 or more than fit: as many as fit)
    long long n_on = 0;     // switched-on workgroups of the march (0: not known)
    int chunk = 0;          // listed steps per staged chunk: 1, 2, or 0 = p3d_list_chunk's rule
    // the queue leaves the outputs of switched-off workgroups unwritten; without the fused primal step
    // it is used only when the caller never reads them (off_unread)
    bool off_unread = false;
};
int launch_project_t(sipo_plan p, const void *vol_t, void *sino_t, hipStream_t s, const uint8_t *wg_on = nullptr,
                     const SplitSpec &sp = SplitSpec(), const PrimalFuse *fuse = nullptr,
                     const StepList &sl = StepList());
// Step lists of an LP solve: a workgroup of the projector (at the plan's current slices per thread)
// lists the march steps whose staged strip holds a voxel within the PSF box of a labelled voxel in
// one of its slices (K z vanishes elsewhere, since z does off the labelled voxels); workgroups whose
// flag is off list none.  labels: [z][y][x]; reach: scratch of p3d_reach_bytes; steps: int
// [p3d_flag_count][n]; count: int [p3d_flag_count].  Needs the asynchronous projector's ranges.
bool p3d_steps_ok(sipo_plan p);   // the plan's projector (current tuning) can walk step lists
// Listed march steps per staged chunk of the projector on these lists: 1 at 32 slices per thread;
// else sl.chunk if set; else 2 when all sl.n_on switched-on workgroups fit on the device at once
// with the two-step ring, 1 otherwise.  The sums are the same either way (steps in list order).
int p3d_list_chunk(sipo_plan p, const StepList &sl);
size_t p3d_reach_bytes(sipo_plan p, int zc = 0);
int launch_p3d_steps(sipo_plan p, const uint8_t *labels, const uint8_t *wg_on, uint8_t *reach, int *steps, int *count,
                     hipStream_t s);
// projector workgroups / backprojector tiles of a fast3d plan (else 0) at zc slices per thread
// (zc <= 0: the plan's current tuning)
size_t p3d_flag_count(sipo_plan p, int zc = 0);
size_t bp3d_flag_count(sipo_plan p, int zc = 0);
// Bytes of the backprojector's per-column need mask at zc slices per thread (0 = the plan's), and
// its builder (scratch: as many bytes, overwritten).
size_t bp3d_need_bytes(sipo_plan p, int zc = 0);
int launch_bp3d_need(sipo_plan p, const uint8_t *labels, uint8_t *scratch, uint8_t *need, hipStream_t s);
int launch_p3d_flags(sipo_plan p, const uint8_t *act_t, uint8_t *flags, hipStream_t s);
int launch_bp3d_flags(sipo_plan p, const uint8_t *labels, uint8_t *flags, hipStream_t s);
// tile_on: optional flags per 16 (z) x 256 (y n + x) tile of the volume (see vol_t_tile_count);
// tiles that are off are not written
int launch_vol_to_t(sipo_plan p, const void *vol, void *vol_t, hipStream_t s, const uint8_t *tile_on = nullptr);
size_t vol_t_tile_count(sipo_plan p);
constexpr int kTrRows = 16, kTrCols = 256;   // tile of the flagged transpose: slices x (y n + x) columns
// Transpose tiles holding a voxel of a blur tile flagged in `reach` (flags of blur_tile_count
// at the plan's current blur tuning): elsewhere the blurred field is zero.
int launch_vol_t_flags(sipo_plan p, const uint8_t *reach, uint8_t *tflags, hipStream_t s);
int launch_sino_to_t(sipo_plan p, const void *sino, void *sino_t, hipStream_t s);
int launch_sino_from_t(sipo_plan p, const void *sino_t, void *sino, int accumulate, hipStream_t s);
int launch_mask_to_t(sipo_plan p, const uint8_t *mask, uint8_t *mask_t, hipStream_t s);
int plan_build_batches(sipo_plan p, const double2 *trig_host);
constexpr int kPB = 32, kPV = 8, kPCM = 4, kPCR = 96;   // bins, views, steps per stage, max staged cross range

// 2D (single-slice) operators, batched over instances.  One Geo2D describes an
// instance: its plan's tables and where its arrays sit in packed sinogram and
// volume arrays (element offsets).  Work items are int4 records.
struct Geo2D {
    const double2 *trig;     // [n_angles] (sin, cos)
    const int *walk;         // walked views (first of each opposite pair when pair != 0)
    const int *partner;      // [n_angles] opposite view or -1
    long long soff, voff;    // offsets of the instance's sinogram / volume
    int n, n_angles, n_bins, n_walk;
    int pair, nc;            // views walked in opposite pairs; candidate voxels per ray step
    double h, inv_ds, atten;
    const int2 *vial;        // [n]: first and last index along a grid line inside the vial
};
// Work shapes of the 2D pair (256 threads per workgroup): P^T tiles of bx x by voxels with vb walked
// views staged per batch, P bundles of fb bins x 256 / fb walked views.  The defaults serve every
// plan; the other shapes exist for FP32 staged launches (the batched solver's tuner picks them).
struct Tiles2D {
    int bx = 32, by = 8, vb = 16, fb = 64;
    int fv() const { return 256 / fb; }
    bool is_default() const { return bx == 32 && by == 8 && vb == 16 && fb == 64; }
    bool operator==(const Tiles2D &o) const { return bx == o.bx && by == o.by && vb == o.vb && fb == o.fb; }
};
bool tiles2d_valid(const Tiles2D &t);
Geo2D plan_geo2d(sipo_plan p, long long soff, long long voff);
// Items of one instance appended to a list: P^T (geo, x0, y0, 0) and P (geo, first walked view, b0, 0).
void append_items_bp2d(const Geo2D &g, int geo_index, std::vector<int4> &items, const Tiles2D &t = Tiles2D());
void append_items_fp2d(const Geo2D &g, int geo_index, std::vector<int4> &items, const Tiles2D &t = Tiles2D());
bool bp2d_stage_fits(int n, int n_bins, const Tiles2D &t = Tiles2D());
int launch_bp2d(sipo_dtype dt, bool staged, const Geo2D *geo, const int4 *items, int n_items, const void *sino,
                void *vol, int accumulate, hipStream_t s, const Tiles2D &t = Tiles2D());
// vol_xt: optional [x][y] copy of the volume (from launch_tr2d), read by rays that march along x
constexpr int kF2MaxN = 16384;   // largest single-slice grid of the 2D projector (its LDS holds n vial extents)
int launch_fp2d(sipo_dtype dt, int nc, int n_max, const Geo2D *geo, const int4 *items, int n_items, const void *vol,
                const void *vol_xt, void *sino, int accumulate, hipStream_t s, const Tiles2D &t = Tiles2D());
// Per-instance transpose of single-slice volumes: out[x][y] = in[y][x]; items (geo, x0, y0, 0) of 64 x 64 tiles.
void append_items_tr2d(const Geo2D &g, int geo_index, std::vector<int4> &items);
int launch_tr2d(sipo_dtype dt, const Geo2D *geo, const int4 *items, int n_items, const void *in, void *out,
                hipStream_t s);
int plan_build_2d(sipo_plan p);

// ------------------------------------------------------------- geometry
// The per-(voxel, view) interpolation taps, shared verbatim by the
// backprojector and the projector so that the two are exact transposes.
// Position and detector coordinate are evaluated in double precision; the
// Beer-Lambert factor in the element type.
__device__ __forceinline__ double centre(int c, double h) { return fma((double)c + 0.5, h, -1.0); }

// exp(-k v) and sqrt: the FP32 path uses the hardware v_exp_f32 / v_sqrt_f32
// (about 1 ulp), the FP64 path the correctly rounded library functions.
constexpr double kLog2e = 1.4426950408889634;

template <typename T>
__device__ __forceinline__ T exp_neg(T k, T v);   // exp(-k v)
template <>
__device__ __forceinline__ float exp_neg<float>(float k, float v) {
    return __builtin_amdgcn_exp2f(-(k * (float)kLog2e) * v);
}
template <>
__device__ __forceinline__ double exp_neg<double>(double k, double v) { return exp(-k * v); }

template <typename T>
__device__ __forceinline__ T sqrt_t(T v);
template <>
__device__ __forceinline__ float sqrt_t<float>(float v) { return __builtin_amdgcn_sqrtf(v); }
template <>
__device__ __forceinline__ double sqrt_t<double>(double v) { return sqrt(v); }

// Returns b = floor(u); w0 = a (1 - f) belongs to bin b and w1 = a f to bin b+1.
template <typename T>
__device__ __forceinline__ int taps(double x, double y, double sn, double cs, double inv_ds, T atten,
                                    T &w0, T &w1) {
#pragma clang fp contract(off)
    const double s = fma(-x, sn, y * cs);
    const double u = fma(s + 1.0, inv_ds, -0.5);
    const double bf = floor(u);
    const T f = (T)(u - bf);
    const double t = fma(x, cs, y * sn);
    T r = (T)fma(-s, s, 1.0);
    r = r > (T)0 ? sqrt_t<T>(r) : (T)0;
    const T a = exp_neg<T>(atten, (T)t + r);
    w1 = a * f;
    w0 = a - w1;
    return (int)bf;
}

// ------------------------------------------------ FP32 detector coordinates
// The FP32 kernels evaluate the detector coordinate u (and the position of a voxel in a ray's hat
// function) without FP64 in their inner loops.  A per-(tile, view) or per-ray origin and the
// coordinate's increments are formed in FP64 once, then each is split into hi = the value rounded to
// a multiple of 2^-q and lo = the rest, both FP32.  Sums of hi parts with small integer multipliers
// are exact in FP32 while they stay below 2^(24 - q) (every such sum is a multiple of 2^-q), and the lo
// parts are small enough that their FP32 rounding is far below 1e-7, so the fractional part that
// weights the interpolation taps comes out with an absolute error near 1e-7 whatever the grid size.
struct Split32 {
    float hi, lo;
};
__device__ __forceinline__ Split32 split32(double v, double scale, double inv_scale) {
    const double h = rint(v * scale) * inv_scale;
    return {(float)h, (float)(v - h)};
}

// floor and fraction of hi + lo, where hi is an exact multiple of 2^-q and |lo| < 1:
// returns b with hi + lo = b + f, 0 <= f < 1 (f to about 1e-7)
__device__ __forceinline__ int floor_frac(float hi, float lo, float &f) {
    const float bh = floorf(hi);
    float fr = (hi - bh) + lo;          // hi - bh is exact
    int b = (int)bh;
    if (fr < 0.f) { fr += 1.f; --b; }
    if (fr >= 1.f) { fr -= 1.f; ++b; }
    f = fr;
    return b;
}

// Taps of a voxel at integer offsets (dc, dr) from its tile's origin, relative to the tile's first
// staged bin: u - bm = u0 + dc du_dc + dr du_dr with the three terms split as above (q = 16: the
// relative coordinate stays below 128).  Returns the bin index relative to bm; w0 = a (1 - f) belongs
// to it, w1 = a f to the next bin; s and t are the voxel's detector and depth coordinates.
__device__ __forceinline__ int taps_rel32(float dc, float dr, const Split32 &u0, const Split32 &ux, const Split32 &uy,
                                          float s, float t, float atten, float &w0, float &w1) {
    const float hi = fmaf(dr, uy.hi, fmaf(dc, ux.hi, u0.hi));   // exact
    const float lo = fmaf(dr, uy.lo, fmaf(dc, ux.lo, u0.lo));
    float f;
    const int b = floor_frac(hi, lo, f);
    float r = fmaf(-s, s, 1.f);
    r = r > 0.f ? sqrt_t<float>(r) : 0.f;
    const float a = exp_neg<float>(atten, t + r);
    w1 = a * f;
    w0 = a - w1;
    return b;
}
constexpr double kTapScale = 65536.0, kTapInvScale = 1.0 / 65536.0;   // q = 16

// A ray's march in FP32.  Along grid line m the ray's hat position of the voxel at cross index j is
// d = w(m) + j du with w(m) = U00 - b + m dU (b the ray's bin); its detector and depth coordinates
// are s00 + m dsm + j dsj and t00 + m dtm + j dtj.  w's origin and both steps are split at 2^-q with
// q = 20 - floor(log2(n_bins)) (in [4, 16]): the hi parts of w and d then stay below 2^(24 - q), so
// they are exact, and d, which lies in [-1, 1], keeps an absolute error near 1e-7.  The first
// candidate jlo comes from w rounded to FP32; near a hat edge it may be off by one, which drops or
// adds only a voxel whose weight is below that rounding (about 1e-4 at 512 bins), and the candidate
// count (at least 2 / |du|) still covers the rest.
struct MarchF32 {
    Split32 w0, dU, du;
    float inv_du, s00, dsm, t00, dtm;
};
__device__ __forceinline__ MarchF32 march_f32(double w0, double dU, double du, double inv_du, double s00, double dsm,
                                              double t00, double dtm, int nb) {
    const int q = min(16, max(4, 20 - (31 - __clz(max(nb, 1)))));
    const double qs = ldexp(1.0, q), qi = ldexp(1.0, -q);
    MarchF32 r;
    r.w0 = split32(w0, qs, qi);
    r.dU = split32(dU, qs, qi);
    r.du = split32(du, qs, qi);
    r.inv_du = (float)inv_du;
    r.s00 = (float)s00; r.dsm = (float)dsm; r.t00 = (float)t00; r.dtm = (float)dtm;
    return r;
}
// First candidate of grid line m, its hat position d0 and coordinates s0, t0 (FP32 only).
template <typename T>
__device__ __forceinline__ int march_step_f32(const MarchF32 &c, int m, T dsj, T dtj, T &d0, T &s0, T &t0) {
    const float mf = (float)m;
    const float whi = fmaf(mf, c.dU.hi, c.w0.hi), wlo = fmaf(mf, c.dU.lo, c.w0.lo);   // whi exact
    const float wf = whi + wlo;
    const int jlo = (int)ceilf(fminf((-1.f - wf) * c.inv_du, (1.f - wf) * c.inv_du));
    const float jl = (float)jlo;
    d0 = fmaf(jl, c.du.hi, whi) + fmaf(jl, c.du.lo, wlo);   // the first product-sum is exact
    s0 = fmaf(jl, (float)dsj, fmaf(mf, c.dsm, c.s00));
    t0 = fmaf(jl, (float)dtj, fmaf(mf, c.dtm, c.t00));
    return jlo;
}

}  // namespace sipo
