// C-ABI entry points: error reporting, plans and argument validation for the
// operator calls.  Kernels live in projector.hip, blur.hip, regions.hip and
// pdhg.hip.
#include <cstdarg>
#include <cstring>
#include <vector>
#include <algorithm>

#include "sipo_internal.hpp"

namespace sipo {

static thread_local char g_err[1024] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int check_plan(sipo_plan p) {
    SIPO_REQUIRE(p != nullptr, "plan is NULL");
    int dev = -1;
    SIPO_HIP(hipGetDevice(&dev));
    SIPO_REQUIRE(dev == p->device, "plan was created on device %d but device %d is current", p->device, dev);
    return SIPO_OK;
}

int check_plan_ws(sipo_plan p) {
    if (!p->ws)
        return fail(SIPO_E_WORKSPACE, "this call needs the plan's workspace: attach %zu bytes of device memory with "
                    "sipo_plan_set_workspace", p->ws_need());
    if (p->ws_bytes < p->ws_need())
        return fail(SIPO_E_WORKSPACE, "plan workspace of %zu bytes is smaller than the %zu bytes needed", p->ws_bytes,
                    p->ws_need());
    return SIPO_OK;
}

int plan_alloc(sipo_plan p, void **ptr, size_t bytes) {
    *ptr = nullptr;
    SIPO_HIP(hipMalloc(ptr, bytes));
    p->table_bytes += bytes;
    return SIPO_OK;
}

template <typename T>
static int fill_taps(Taps<T> &t, const sipo_psf *psf) {
    std::memset(&t, 0, sizeof(t));
    t.kx[0] = t.ky[0] = t.kz[0] = (T)1;
    if (!psf) return SIPO_OK;
    const int r[3] = {psf->rx, psf->ry, psf->rz};
    const double *k[3] = {psf->kx, psf->ky, psf->kz};
    T *dst[3] = {t.kx, t.ky, t.kz};
    for (int a = 0; a < 3; ++a) {
        SIPO_REQUIRE(r[a] >= 0 && r[a] <= kMaxR, "PSF radius %d outside [0, %d]", r[a], kMaxR);
        if (r[a] == 0 && k[a] == nullptr) { dst[a][0] = (T)1; continue; }
        SIPO_REQUIRE(k[a] != nullptr, "PSF taps pointer for axis %d is NULL", a);
        for (int i = 0; i <= 2 * r[a]; ++i) {
            SIPO_REQUIRE(std::isfinite(k[a][i]), "PSF tap %d of axis %d is not finite", i, a);
            dst[a][i] = (T)k[a][i];
        }
    }
    t.rx = r[0]; t.ry = r[1]; t.rz = r[2];
    return SIPO_OK;
}

}  // namespace sipo

using namespace sipo;

extern "C" {

const char *sipo_last_error(void) { return g_err; }

const char *sipo_version(void) { return "sipo-mi355x 0.1 (gfx950)"; }

int sipo_plan_create(const sipo_geometry *geom, const sipo_psf *psf, sipo_dtype dtype, sipo_plan *plan_out) {
    SIPO_REQUIRE(geom != nullptr && plan_out != nullptr, "geometry or output pointer is NULL");
    *plan_out = nullptr;
    SIPO_REQUIRE(geom->n >= 1 && geom->nz >= 1 && geom->n_angles >= 1 && geom->n_bins >= 1,
                 "sizes must be >= 1 (n=%d nz=%d n_angles=%d n_bins=%d)", geom->n, geom->nz, geom->n_angles,
                 geom->n_bins);
    SIPO_REQUIRE(geom->n <= 16384 && geom->n_bins <= 16384 && geom->n_angles <= 65535 && geom->nz <= 16384,
                 "sizes exceed the supported maximum");
    SIPO_REQUIRE(geom->angles != nullptr, "angles pointer is NULL");
    SIPO_REQUIRE(std::isfinite(geom->atten) && geom->atten >= 0.0, "atten must be finite and >= 0");
    SIPO_REQUIRE(dtype == SIPO_F32 || dtype == SIPO_F64, "unknown dtype %d", (int)dtype);
    for (int a = 0; a < geom->n_angles; ++a)
        SIPO_REQUIRE(std::isfinite(geom->angles[a]), "angle %d is not finite", a);

    sipo_plan_s *p = new (std::nothrow) sipo_plan_s();
    if (!p) return fail(SIPO_E_DEVICE, "host allocation failed");
    p->n = geom->n; p->nz = geom->nz; p->n_angles = geom->n_angles; p->n_bins = geom->n_bins;
    p->atten = geom->atten; p->dtype = dtype; p->has_psf = psf != nullptr;
    int rc = fill_taps(p->taps_f, psf);
    if (rc == SIPO_OK) rc = fill_taps(p->taps_d, psf);
    if (rc != SIPO_OK) { delete p; return rc; }
    if (hipGetDevice(&p->device) != hipSuccess) { delete p; return fail(SIPO_E_DEVICE, "hipGetDevice failed"); }

    std::vector<double2> trig(geom->n_angles);
    std::vector<int> order;
    order.reserve(geom->n_angles);
    for (int a = 0; a < geom->n_angles; ++a) {
        trig[a] = make_double2(std::sin(geom->angles[a]), std::cos(geom->angles[a]));
        if (std::fabs(trig[a].y) >= std::fabs(trig[a].x)) order.push_back(a);
    }
    p->n_xmajor = (int)order.size();
    for (int a = 0; a < geom->n_angles; ++a)
        if (!(std::fabs(trig[a].y) >= std::fabs(trig[a].x))) order.push_back(a);

    rc = plan_alloc(p, (void **)&p->d_trig, sizeof(double2) * geom->n_angles);
    if (rc == SIPO_OK) rc = plan_alloc(p, (void **)&p->d_angle_order, sizeof(int) * geom->n_angles);
    hipError_t e = hipSuccess;
    if (rc == SIPO_OK) e = hipMemcpy(p->d_trig, trig.data(), sizeof(double2) * geom->n_angles, hipMemcpyHostToDevice);
    if (rc == SIPO_OK && e == hipSuccess)
        e = hipMemcpy(p->d_angle_order, order.data(), sizeof(int) * geom->n_angles, hipMemcpyHostToDevice);
    if (rc != SIPO_OK || e != hipSuccess) {
        (void)hipFree(p->d_trig); (void)hipFree(p->d_angle_order);
        delete p;
        return rc != SIPO_OK ? rc : fail(SIPO_E_DEVICE, "plan table upload failed: %s", hipGetErrorString(e));
    }
    p->d_batches = nullptr;
    p->d_partner = nullptr;
    p->d_view_batch = nullptr;
    p->d_ranges = nullptr;
    p->d_vial_rows = nullptr;
    p->d_zero = nullptr;
    p->d_geo2d = nullptr;
    p->d_items_bp2d = p->d_items_fp2d = p->d_items_tr2d = nullptr;
    p->n_items_bp2d = p->n_items_fp2d = p->n_items_tr2d = 0;
    p->p2d_ok = false;
    p->ws = nullptr;
    p->ws_bytes = 0;
    rc = plan_build_batches(p, trig.data());
    if (rc == SIPO_OK) rc = plan_build_2d(p);
    if (rc != SIPO_OK) {
        (void)hipFree(p->d_trig); (void)hipFree(p->d_angle_order);
        (void)hipFree(p->d_batches);
        (void)hipFree(p->d_partner);
        (void)hipFree(p->d_view_batch);
        (void)hipFree(p->d_ranges);
        (void)hipFree(p->d_vial_rows);
        (void)hipFree(p->d_zero);
        (void)hipFree(p->d_geo2d);
        (void)hipFree(p->d_items_bp2d);
        (void)hipFree(p->d_items_fp2d);
        (void)hipFree(p->d_items_tr2d);
        delete p;
        return rc;
    }
    *plan_out = p;
    return SIPO_OK;
}

int sipo_plan_destroy(sipo_plan p) {
    if (!p) return SIPO_OK;
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != p->device) (void)hipSetDevice(p->device);
    (void)hipFree(p->d_trig);
    (void)hipFree(p->d_angle_order);
    (void)hipFree(p->d_batches);
    (void)hipFree(p->d_partner);
    (void)hipFree(p->d_view_batch);
    (void)hipFree(p->d_ranges);
    (void)hipFree(p->d_vial_rows);
    (void)hipFree(p->d_zero);
    (void)hipFree(p->d_geo2d);
    (void)hipFree(p->d_items_bp2d);
    (void)hipFree(p->d_items_fp2d);
    (void)hipFree(p->d_items_tr2d);
    if (cur >= 0 && cur != p->device) (void)hipSetDevice(cur);
    delete p;
    return SIPO_OK;
}

size_t sipo_plan_workspace_size(sipo_plan plan) { return plan ? plan->ws_need() : 0; }

size_t sipo_plan_device_bytes(sipo_plan plan) { return plan ? plan->table_bytes : 0; }

int sipo_plan_set_workspace(sipo_plan plan, void *workspace, size_t bytes) {
    int rc = check_plan(plan);
    if (rc) return rc;
    if (!workspace) {
        plan->ws = nullptr;
        plan->ws_bytes = 0;
        return SIPO_OK;
    }
    SIPO_REQUIRE(((uintptr_t)workspace & 255) == 0, "plan workspace must be 256-byte aligned");
    if (bytes < plan->ws_need())
        return fail(SIPO_E_WORKSPACE, "plan workspace of %zu bytes is smaller than the %zu bytes needed", bytes,
                    plan->ws_need());
    plan->ws = workspace;
    plan->ws_bytes = bytes;
    return SIPO_OK;
}

int sipo_backproject(sipo_plan plan, const void *sino, void *vol, int accumulate, void *stream) {
    int rc = check_plan(plan);
    if (rc) return rc;
    SIPO_REQUIRE(sino && vol, "sino or vol is NULL");
    const char *s0 = (const char *)sino, *v0 = (const char *)vol;
    const size_t sb = plan->sino_elems() * plan->elem_bytes(), vb = plan->vol_elems() * plan->elem_bytes();
    SIPO_REQUIRE(s0 + sb <= v0 || v0 + vb <= s0, "sino and vol overlap");
    return launch_backproject(plan, sino, vol, accumulate, (hipStream_t)stream);
}

int sipo_project(sipo_plan plan, const void *vol, void *sino, int accumulate, void *stream) {
    int rc = check_plan(plan);
    if (rc) return rc;
    SIPO_REQUIRE(sino && vol, "sino or vol is NULL");
    const char *s0 = (const char *)sino, *v0 = (const char *)vol;
    const size_t sb = plan->sino_elems() * plan->elem_bytes(), vb = plan->vol_elems() * plan->elem_bytes();
    SIPO_REQUIRE(s0 + sb <= v0 || v0 + vb <= s0, "sino and vol overlap");
    return launch_project(plan, vol, sino, accumulate, (hipStream_t)stream);
}

int sipo_blur(sipo_plan plan, const void *in, void *out, void *stream) {
    int rc = check_plan(plan);
    if (rc) return rc;
    SIPO_REQUIRE(in && out, "in or out is NULL");
    const size_t vb = plan->vol_elems() * plan->elem_bytes();
    const char *a = (const char *)in, *b = (const char *)out;
    SIPO_REQUIRE(a + vb <= b || b + vb <= a, "in and out overlap");
    return launch_blur(plan, in, out, (hipStream_t)stream);
}

}  // extern "C"
