// Plan autotuner: picks, per plan, the fastest of the kernel variants that
// compute the same operator with different work splits.
#include <vector>

#include "sipo_internal.hpp"

namespace sipo {

// Mean time of reps launches of fn after one warm-up launch (ms), or < 0 on error.
template <typename F>
static float time_ms(F fn, int reps, hipStream_t s) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.f;
    float ms = -1.f;
    if (fn() == SIPO_OK && hipEventRecord(e0, s) == hipSuccess) {
        bool ok = true;
        for (int r = 0; r < reps && ok; ++r) ok = fn() == SIPO_OK;
        if (ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
            hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
            ms /= (float)reps;
        else
            ms = -1.f;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
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
    constexpr int kReps = 3;
    if (p->fast3d()) {
        std::vector<int> zcs = p->dtype == SIPO_F64 ? std::vector<int>{8, 16} : std::vector<int>{16, 32};
        int best = p->p3d_zc;
        bool best_dma = p->p3d_dma, best_skip = p->p3d_skip;
        float tbest = 1e30f;
        for (int dma = 0; dma <= (p->p3d_dma_ok ? 1 : 0); ++dma)
            for (int skip = 0; skip <= dma; ++skip)
                for (int zc : zcs) {
                    p->p3d_zc = zc;
                    p->p3d_dma = dma != 0;
                    p->p3d_skip = skip != 0;
                    const float t = time_ms([&] { return launch_project_t(p, va, sa, s); }, kReps, s);
                    if (t >= 0.f && t < tbest) { tbest = t; best = zc; best_dma = dma != 0; best_skip = skip != 0; }
                }
        p->p3d_zc = best;
        p->p3d_dma = best_dma;
        p->p3d_skip = best_skip;
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
