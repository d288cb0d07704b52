// Level schedule of a plan and its execution on a HIP stream.
//
// One level (paper Sec. 2.2): u = dx0^2 * G * f on the level's blocks, one
// blockwise convolution per component.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "lgf_runtime.hpp"

namespace lgf {

void build_schedule(lgf_plan *p) {
    if (p->K != 1) throw Failure(LGF_E_UNSUPPORTED, "composite (K > 1) plans are not served by this build yet");
    if (p->prec != LGF_FP64) throw Failure(LGF_E_UNSUPPORTED, "LGF_FP32_REFINE is not served by this build yet");
    auto c = std::make_unique<Conv>();
    build_conv(p, *c, p->levels[0], p->levels[0], false);
    p->convs.push_back(std::move(c));
    plan_alloc_spectral(p);
}

static void enqueue(lgf_plan *p, const double *f, double *u, hipStream_t s) {
    const Conv &c = *p->convs[0];
    for (int comp = 0; comp < p->nc; ++comp)
        run_conv(p, c, f + (size_t)comp * p->comp_len, u + (size_t)comp * p->comp_len, p->dx0, 0, s);
}

void run_plan(lgf_plan *p, const double *f, double *u, hipStream_t s, lgf_report *rep) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rep) {
        hip_check(hipEventCreate(&e0), "event");
        hip_check(hipEventCreate(&e1), "event");
        hip_check(hipEventRecord(e0, s), "event record");
    }
    enqueue(p, f, u, s);
    if (rep) {
        hip_check(hipEventRecord(e1, s), "event record");
        hip_check(hipEventSynchronize(e1), "event sync");
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
        rep->device_ms = ms;
        rep->refine_rel_l2 = 0.0;
        rep->passes = 1;
        hipEventDestroy(e0);
        hipEventDestroy(e1);
    }
}

void run_batch(lgf_context *ctx, int n, lgf_plan *const *plans, const double *const *f, double *const *u,
               hipStream_t s, lgf_report *reps) {
    (void)ctx;
    for (int i = 0; i < n; ++i) run_plan(plans[i], f[i], u[i], s, reps ? &reps[i] : nullptr);
}

}  // namespace lgf
