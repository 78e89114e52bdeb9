// Dual evaluation that allocates nothing, for callers that cannot allocate
// device memory (code under stream capture, tight serving loops).
//
// The evaluation's work-item partials (per-item log-sum-exp and kept-pair
// partials of the objective pass, per-item target sums of the gradient pass)
// live in `scratch`, a file-scope device array of RSOT_NOALLOC_SCRATCH_BYTES
// that every device the library runs on holds until the process ends. Its
// device address is taken once per device with hipGetSymbolAddress, with that
// device current; host code never passes the array's own name to a kernel
// (on the host it is only a stand-in for the symbol). Every partial is written
// before it is read, so nothing needs clearing between calls; calls that
// overlap on one device share the array and race.
#include <mutex>

#include "rsot_internal.h"

#define RSOT_NOALLOC_SCRATCH_BYTES (size_t(64) << 20)

static __device__ __align__(256) double scratch[RSOT_NOALLOC_SCRATCH_BYTES / sizeof(double)];

static std::mutex g_scratch_mu;
static double *g_scratch_ptr[64];

// device address of this device's copy of `scratch` (current device)
static rsot_status scratch_on_device(double **out) {
    int dev = -1;
    RSOT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return RSOT_ERR_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return RSOT_ERR_DEVICE;
        g_scratch_ptr[dev] = (double *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return RSOT_OK;
}

extern "C" rsot_status rsot_dual_eval_noalloc(rsot_problem *p, double eps, const double *psi,
                                              double *J_out, double *grad_out,
                                              rsot_eval_info *info) {
    if (!p || !psi || !J_out) return RSOT_ERR_INVALID_ARG;
    if (p->opt.cost_kind != RSOT_COST_SQEUCLID) return RSOT_ERR_INVALID_ARG;
    if (!(eps > 0.0) || !std::isfinite(eps)) return RSOT_ERR_INVALID_ARG;
    if (p->opt.truncation != RSOT_TRUNC_DENSE) return RSOT_ERR_INVALID_ARG;
    double *s = nullptr;
    RSOT_TRY(scratch_on_device(&s));
    return rsot_eval_dense_in(p, eps, psi, J_out, grad_out, info, s, RSOT_NOALLOC_SCRATCH_BYTES);
}
