// Autotuning of the tile plan: elements per workgroup (the tile size), the element order
// of the tiles (locality order or input order), or no tiles at all (the per-element
// scatter, no LDS combining).  Each candidate's pattern is built and its assembly timed
// with HIP events on the caller's stream; the caller keeps the result (the Python layer
// keeps a JSON cache keyed by architecture, form, element kind and size).
#include <vector>

#include "fem_internal.h"

using namespace fem;

extern "C" {

int fem_autotune(const fem_mesh *mesh, int32_t ncomp, const fem_form *form, const double *coef,
                 unsigned assemble_flags, int32_t n_candidates, const unsigned *build_flags,
                 const unsigned *extra_flags, int32_t reps, double *ms, int32_t *best,
                 void *stream)
{
    clear_error();
    TraceRange trace_range("fem_autotune");
    FEM_TRY(check_mesh(mesh, true));
    if (!form) return fail(FEM_ERR_INVALID_ARG, "form is NULL");
    if (n_candidates <= 0 || !build_flags || !ms || !best)
        return fail(FEM_ERR_INVALID_ARG, "candidates, ms and best are required");
    if (reps <= 0) return fail(FEM_ERR_INVALID_ARG, "reps must be positive");
    if (assemble_flags & FEM_ACCUMULATE)
        return fail(FEM_ERR_INVALID_ARG, "timing runs overwrite; FEM_ACCUMULATE is not taken");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    FEM_HIP_TRY(hipEventCreate(&e0));
    FEM_HIP_TRY(hipEventCreate(&e1));
    *best = -1;
    int rc = FEM_OK;
    for (int32_t c = 0; c < n_candidates && rc == FEM_OK; ++c) {
        ms[c] = -1.0;
        fem_pattern *p = nullptr;
        // a candidate the plan cannot take (a tile size out of range, LDS) is skipped
        if (fem_build_pattern(mesh, ncomp, build_flags[c], &p, stream) != FEM_OK) {
            clear_error();
            continue;
        }
        double *buf = nullptr;
        const size_t bytes = sizeof(double) * (size_t)(p->nnz + p->n_rows + 2);
        if (hipMallocAsync((void **)&buf, bytes, s) != hipSuccess) {
            fem_pattern_destroy(p);
            rc = fail(FEM_ERR_OOM, "autotune: output allocation failed");
            break;
        }
        double *values = buf, *rhs = buf + p->nnz + 1;
        const unsigned af = assemble_flags | (extra_flags ? extra_flags[c] : 0u);
        int arc = fem_assemble(p, mesh, form, coef, values, rhs, af, stream);
        if (arc == FEM_OK) {
            (void)hipEventRecord(e0, s);
            for (int r = 0; r < reps && arc == FEM_OK; ++r)
                arc = fem_assemble(p, mesh, form, coef, values, rhs, af, stream);
            (void)hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) != hipSuccess) arc = FEM_ERR_HIP;
            float t = 0.0f;
            if (arc == FEM_OK && hipEventElapsedTime(&t, e0, e1) == hipSuccess) {
                ms[c] = (double)t / reps;
                if (*best < 0 || ms[c] < ms[*best]) *best = c;
            }
        }
        (void)hipFreeAsync(buf, s);
        (void)hipStreamSynchronize(s);
        fem_pattern_destroy(p);
        if (arc != FEM_OK && arc != FEM_ERR_UNSUPPORTED) rc = arc;  // a real failure stops
        else clear_error();
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == FEM_OK && *best < 0) rc = fail(FEM_ERR_UNSUPPORTED, "autotune: no candidate ran");
    return rc;
}

}  // extern "C"
