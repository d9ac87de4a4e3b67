// Plan autotuner: picks, per plan, the fastest of the kernel variants that
// compute the same operator with different work splits.
#include <vector>

#include "sipo_internal.hpp"

namespace sipo {

// Shortest of reps timed launches of fn after two warm-up launches (ms), or < 0 on error.  The
// minimum is robust against a GPU that is still raising its clocks when the autotuner starts.
template <typename F>
static float time_ms(F fn, int reps, hipStream_t s) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.f;
    float best = -1.f;
    if (fn() == SIPO_OK && fn() == SIPO_OK) {
        for (int r = 0; r < reps; ++r) {
            float ms = 0.f;
            if (hipEventRecord(e0, s) != hipSuccess || fn() != SIPO_OK || hipEventRecord(e1, s) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                best = -1.f;
                break;
            }
            if (best < 0.f || ms < best) best = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

}  // namespace sipo

using namespace sipo;

extern "C" int sipo_plan_autotune(sipo_plan p, void *stream) {
    int rc = check_plan(p);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const size_t vb = p->vol_elems() * p->elem_bytes(), sb = p->sino_elems() * p->elem_bytes();
    void *va = nullptr, *vc = nullptr, *sa = nullptr;
    hipError_t e = hipMalloc(&va, vb);
    if (e == hipSuccess) e = hipMalloc(&vc, vb);
    if (e == hipSuccess) e = hipMalloc(&sa, sb);
    if (e == hipSuccess) e = hipMemsetAsync(va, 0, vb, s);
    if (e != hipSuccess) {
        (void)hipFree(va); (void)hipFree(vc); (void)hipFree(sa);
        return fail(SIPO_E_DEVICE, "autotune scratch allocation failed: %s", hipGetErrorString(e));
    }
    constexpr int kReps = 5;
    if (p->fast3d()) {
        // candidates in a fixed preference order; the first within 2 % of the fastest wins, so that
        // near-ties resolve the same way from run to run
        struct Cand { int zc, dma, skip, cm; float t; };
        std::vector<Cand> cands;
        const Cand orig{p->p3d_zc, p->p3d_dma ? 1 : 0, p->p3d_skip ? 1 : 0, p->p3d_cm, 0.f};
        const int orig_b = p->bp3d_zc;
        for (int dma = p->p3d_dma_ok ? 1 : 0; dma >= 0; --dma)
            for (int zc : p->dtype == SIPO_F64 ? std::vector<int>{16, 8} : std::vector<int>{32, 16, 64})
                for (int cm = dma ? 1 : 2; cm <= 2; ++cm)
                    for (int skip = 0; skip <= dma; ++skip) {
                        if (zc > 32 && (!dma || cm > 1)) continue;   // 64 slices: asynchronous, one-step chunks
                        p->p3d_zc = zc;
                        p->p3d_dma = dma != 0;
                        p->p3d_skip = skip != 0;
                        p->p3d_cm = cm;
                        cands.push_back({zc, dma, skip, cm, time_ms([&] { return launch_project_t(p, va, sa, s); }, kReps, s)});
                    }
        float tmin = 1e30f;
        for (const Cand &c : cands) if (c.t >= 0.f) tmin = std::min(tmin, c.t);
        p->p3d_zc = orig.zc; p->p3d_dma = orig.dma != 0; p->p3d_skip = orig.skip != 0; p->p3d_cm = orig.cm;
        for (const Cand &c : cands)
            if (c.t >= 0.f && c.t <= 1.02f * tmin) {
                p->p3d_zc = c.zc; p->p3d_dma = c.dma != 0; p->p3d_skip = c.skip != 0; p->p3d_cm = c.cm;
                break;
            }
        std::vector<std::pair<int, float>> bc;
        for (int zc : p->dtype == SIPO_F64 ? std::vector<int>{16, 8} : std::vector<int>{32, 16}) {
            p->bp3d_zc = zc;
            bc.push_back({zc, time_ms([&] { return launch_backproject_t(p, sa, va, 0, s); }, kReps, s)});
        }
        float bmin = 1e30f;
        for (auto &c : bc) if (c.second >= 0.f) bmin = std::min(bmin, c.second);
        p->bp3d_zc = orig_b;
        for (auto &c : bc)
            if (c.second >= 0.f && c.second <= 1.02f * bmin) { p->bp3d_zc = c.first; break; }
    }
    if (p->has_psf && p->nz > 1) {
        int best = 0;
        float tbest = 1e30f;
        for (int zc : {0, 8, 16, 32}) {
            if (zc > p->nz) continue;
            p->blur_zc = zc;
            const float t = time_ms([&] { return launch_blur(p, va, vc, s); }, kReps, s);
            if (t >= 0.f && t < tbest) { tbest = t; best = zc; }
        }
        p->blur_zc = best;
    }
    e = hipStreamSynchronize(s);
    (void)hipFree(va); (void)hipFree(vc); (void)hipFree(sa);
    if (e != hipSuccess) return fail(SIPO_E_DEVICE, "autotune failed: %s", hipGetErrorString(e));
    return SIPO_OK;
}

extern "C" int sipo_plan_get_tuning(sipo_plan p, sipo_tuning *out) {
    int rc = check_plan(p);
    if (rc) return rc;
    SIPO_REQUIRE(out != nullptr, "tuning output is NULL");
    out->p3d_zc = p->p3d_zc;
    out->p3d_dma = p->p3d_dma ? 1 : 0;
    out->p3d_skip = p->p3d_skip ? 1 : 0;
    out->p3d_cm = p->p3d_cm;
    out->blur_zc = p->blur_zc;
    out->bp3d_zc = p->bp3d_zc;
    return SIPO_OK;
}

extern "C" int sipo_plan_set_tuning(sipo_plan p, const sipo_tuning *t) {
    int rc = check_plan(p);
    if (rc) return rc;
    SIPO_REQUIRE(t != nullptr, "tuning is NULL");
    const bool f32 = p->dtype == SIPO_F32;
    SIPO_REQUIRE(t->p3d_zc == 8 || t->p3d_zc == 16 || (f32 && (t->p3d_zc == 32 || t->p3d_zc == 64)),
                 "p3d_zc %d: expected 8 or 16%s", t->p3d_zc, f32 ? ", 32 or 64" : "");
    SIPO_REQUIRE(t->p3d_zc <= 32 || t->p3d_dma, "64 slices per thread need the asynchronous projector");
    SIPO_REQUIRE(t->p3d_dma == 0 || t->p3d_dma == 1, "p3d_dma must be 0 or 1");
    SIPO_REQUIRE(t->p3d_skip == 0 || t->p3d_skip == 1, "p3d_skip must be 0 or 1");
    SIPO_REQUIRE(t->p3d_cm == 1 || t->p3d_cm == 2, "p3d_cm must be 1 or 2");
    SIPO_REQUIRE(t->p3d_zc <= 32 || t->p3d_cm == 1, "64 slices per thread stage one march step per chunk");
    SIPO_REQUIRE(t->blur_zc == 0 || ((t->blur_zc == 8 || t->blur_zc == 16 || t->blur_zc == 32) && t->blur_zc <= p->nz),
                 "blur_zc %d: expected 0, or 8, 16 or 32 not above nz = %d", t->blur_zc, p->nz);
    SIPO_REQUIRE(!t->p3d_skip || t->p3d_dma, "p3d_skip applies to the asynchronous projector only");
    SIPO_REQUIRE(t->bp3d_zc == 4 || t->bp3d_zc == 8 || t->bp3d_zc == 16 || (f32 && t->bp3d_zc == 32),
                 "bp3d_zc %d: expected 4, 8 or 16%s", t->bp3d_zc, f32 ? " or 32" : "");
    if (t->p3d_dma && !p->p3d_dma_ok)
        return fail(SIPO_E_UNSUPPORTED, "the asynchronous 3D projector does not apply to this plan");
    p->p3d_zc = t->p3d_zc;
    p->p3d_dma = t->p3d_dma != 0;
    p->p3d_skip = t->p3d_skip != 0;
    p->p3d_cm = t->p3d_cm;
    p->blur_zc = t->blur_zc;
    p->bp3d_zc = t->bp3d_zc;
    return SIPO_OK;
}

