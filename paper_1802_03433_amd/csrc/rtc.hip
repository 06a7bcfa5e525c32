// Runtime compilation of user integrands (Sec. 5): the caller writes sigma(x) and f(x) as
// C expressions in x, y, z; the library substitutes them into a kernel source template,
// compiles it for the GPU at run time (hipRTC, the HIP counterpart of the NVRTC path the
// paper describes) and runs it.
//
// The generated kernel is the per-element half of Alg. 1: one thread per element reads
// its vertices, forms the geometry, and sums over the points of the chosen rule
//   A_ij += w_q vol (kappa_e grad l_i . sigma(x_q) grad l_j + c l_i(q) l_j(q)),
//   b_i  += w_q vol f(x_q) l_i(q),
// then stores A and b as element matrices ([NP*NP + NP][E], element index fastest).
// The scatter half is the ahead-of-time tile kernel (FEM_FORM_ELEMENT_MATRICES), so a
// compiled form gets every scatter mode of the library.  Rule tables, the dimension and
// the loop bounds are constants of the generated source (the template variables).
#include <hip/hiprtc.h>

#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fem_internal.h"
#include "quadrature.h"

struct fem_rtc {
    int dim = 0, np = 0, nq = 0;
    bool has_load = false;
    std::string source;
    std::vector<char> code;
    std::mutex mu;
    std::map<int, std::pair<hipModule_t, hipFunction_t>> loaded;  // per device
};

namespace fem {
namespace {

template <class R>
void emit_rule(std::string &s, int np)
{
    char buf[64];
    s += "    constexpr double RL[" + std::to_string(R::nq) + "][" + std::to_string(np) + "] = {";
    for (int q = 0; q < R::nq; ++q) {
        s += "{";
        for (int k = 0; k < np; ++k) {
            std::snprintf(buf, sizeof buf, "%.17g%s", R::lam(q, k), k + 1 < np ? ", " : "");
            s += buf;
        }
        s += q + 1 < R::nq ? "}, " : "}";
    }
    s += "};\n    constexpr double RW[" + std::to_string(R::nq) + "] = {";
    for (int q = 0; q < R::nq; ++q) {
        std::snprintf(buf, sizeof buf, "%.17g%s", R::w(q), q + 1 < R::nq ? ", " : "");
        s += buf;
    }
    s += "};\n";
}

std::string make_source(int D, const char *const *sigma, const char *load, int degree, int *nq)
{
    const int NP = D + 1;
    std::string s;
    s += "// generated: P1 element matrices, dim " + std::to_string(D) + "\n";
    s += "extern \"C\" __global__ void fem_rtc_elements(const double *__restrict__ coords, long N,\n"
         "    const int *__restrict__ conn, long E, const double *__restrict__ kappa, double c,\n"
         "    double *__restrict__ out)\n{\n";
    s += "    constexpr int D = " + std::to_string(D) + ", NP = " + std::to_string(NP) + ";\n";
    s += "    const double pi = 3.14159265358979323846;\n";
    if (D == 2) {
        if (degree <= 2) emit_rule<quad::P1Rule<2>>(s, NP), *nq = quad::P1Rule<2>::nq;
        else emit_rule<quad::Tri7>(s, NP), *nq = quad::Tri7::nq;
    } else {
        if (degree <= 2) emit_rule<quad::P1Rule<3>>(s, NP), *nq = quad::P1Rule<3>::nq;
        else emit_rule<quad::Tet14>(s, NP), *nq = quad::Tet14::nq;
    }
    s += "    constexpr int NQ = " + std::to_string(*nq) + ";\n";
    s += R"(    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    double X[NP][D];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const long n = conn[k * E + e];
#pragma unroll
        for (int d = 0; d < D; ++d) X[k][d] = coords[d * N + n];
    }
    double J[D][D];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int m = 0; m < D; ++m) J[a][m] = X[m + 1][a] - X[0][a];
    double inv[D][D], det;
)";
    if (D == 2) {
        s += R"(    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    inv[0][0] = J[1][1] / det; inv[0][1] = -J[0][1] / det;
    inv[1][0] = -J[1][0] / det; inv[1][1] = J[0][0] / det;
    const double vol = 0.5 * fabs(det);
)";
    } else {
        s += R"(    {
        const double C00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        const double C01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        const double C02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        const double C10 = J[0][2] * J[2][1] - J[0][1] * J[2][2];
        const double C11 = J[0][0] * J[2][2] - J[0][2] * J[2][0];
        const double C12 = J[0][1] * J[2][0] - J[0][0] * J[2][1];
        const double C20 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
        const double C21 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
        const double C22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        det = J[0][0] * C00 + J[0][1] * C01 + J[0][2] * C02;
        inv[0][0] = C00 / det; inv[1][0] = C01 / det; inv[2][0] = C02 / det;
        inv[0][1] = C10 / det; inv[1][1] = C11 / det; inv[2][1] = C12 / det;
        inv[0][2] = C20 / det; inv[1][2] = C21 / det; inv[2][2] = C22 / det;
    }
    const double vol = fabs(det) / 6.0;
)";
    }
    s += R"(    double B[NP][D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        double t = 0.0;
#pragma unroll
        for (int m = 0; m < D; ++m) {
            B[m + 1][a] = inv[m][a];
            t += inv[m][a];
        }
        B[0][a] = -t;
    }
    const double kap = kappa[e];
    double A[NP][NP], b[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        b[i] = 0.0;
#pragma unroll
        for (int j = 0; j < NP; ++j) A[i][j] = 0.0;
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double P[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < NP; ++k) t += RL[q][k] * X[k][a];
            P[a] = t;
        }
        const double x = P[0], y = P[1];
)";
    s += D == 3 ? "        const double z = P[2];\n" : "        const double z = 0.0;\n";
    s += "        (void)x; (void)y; (void)z;\n";
    s += "        const double wv = RW[q] * vol;\n";
    if (sigma) {
        s += "        const double S[D][D] = {";
        for (int r = 0; r < D; ++r) {
            s += "{";
            for (int c = 0; c < D; ++c) {
                s += "(double)(";
                s += sigma[r * D + c];
                s += c + 1 < D ? "), " : ")";
            }
            s += r + 1 < D ? "}, " : "}";
        }
        s += "};\n";
    } else {
        s += "        const double S[D][D] = {";
        for (int r = 0; r < D; ++r) {
            s += "{";
            for (int c = 0; c < D; ++c) s += std::string(r == c ? "1.0" : "0.0") + (c + 1 < D ? ", " : "");
            s += r + 1 < D ? "}, " : "}";
        }
        s += "};\n";
    }
    s += R"(        double C[NP][D];  // C = B S
#pragma unroll
        for (int i = 0; i < NP; ++i)
#pragma unroll
            for (int bb = 0; bb < D; ++bb) {
                double t = 0.0;
#pragma unroll
                for (int a = 0; a < D; ++a) t += B[i][a] * S[a][bb];
                C[i][bb] = t;
            }
#pragma unroll
        for (int i = 0; i < NP; ++i)
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                double g = 0.0;
#pragma unroll
                for (int bb = 0; bb < D; ++bb) g += C[i][bb] * B[j][bb];
                A[i][j] += wv * (kap * g + c * RL[q][i] * RL[q][j]);
            }
)";
    if (load) {
        s += "        const double fv = (double)(";
        s += load;
        s += ");\n";
        s += R"(#pragma unroll
        for (int i = 0; i < NP; ++i) b[i] += wv * fv * RL[q][i];
)";
    }
    s += R"(    }
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
        for (int j = 0; j < NP; ++j) out[(long)(i * NP + j) * E + e] = A[i][j];
)";
    if (load)
        s += R"(#pragma unroll
    for (int i = 0; i < NP; ++i) out[(long)(NP * NP + i) * E + e] = b[i];
)";
    s += "}\n";
    return s;
}

// dL/dkappa_e = <Gbar_e, K_e> with K_e the element matrix at kappa = 1, c = 0 (the form
// is linear in kappa): Gbar_e gathered through the element-to-slot map
__global__ void k_rtc_dkappa(const int32_t *__restrict__ slot, int64_t E, int np,
                             const double *__restrict__ K, const double *__restrict__ gvalues,
                             double *__restrict__ gcoef, bool accumulate)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    double s = 0.0;
    for (int t = 0; t < np * np; ++t) s += gvalues[slot[t * E + e]] * K[t * E + e];
    if (accumulate) gcoef[e] += s;
    else gcoef[e] = s;
}

__global__ void k_fill_ones(double *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 1.0;
}

int rtc_function(fem_rtc *r, hipFunction_t *fn)
{
    int dev = 0;
    FEM_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(r->mu);
    auto it = r->loaded.find(dev);
    if (it != r->loaded.end()) {
        *fn = it->second.second;
        return FEM_OK;
    }
    hipModule_t mod;
    FEM_HIP_TRY(hipModuleLoadData(&mod, r->code.data()));
    hipFunction_t f;
    hipError_t e = hipModuleGetFunction(&f, mod, "fem_rtc_elements");
    if (e != hipSuccess) {
        (void)hipModuleUnload(mod);
        return fail(FEM_ERR_HIP, std::string("hipModuleGetFunction: ") + hipGetErrorString(e));
    }
    r->loaded[dev] = {mod, f};
    *fn = f;
    return FEM_OK;
}

}  // namespace
}  // namespace fem

using namespace fem;

extern "C" {

int fem_rtc_compile(int32_t dim, const char *const *sigma, const char *load, int32_t degree,
                    fem_rtc **out)
{
    clear_error();
    TraceRange trace_range("fem_rtc_compile");
    if (!out) return fail(FEM_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (dim != 2 && dim != 3) return fail(FEM_ERR_INVALID_ARG, "dim must be 2 or 3");
    if (degree < 0 || degree > 5) return fail(FEM_ERR_INVALID_ARG, "degree must be 0..5");
    if (sigma)
        for (int k = 0; k < dim * dim; ++k)
            if (!sigma[k]) return fail(FEM_ERR_INVALID_ARG, "a sigma entry is NULL");
    int nq = 0;
    std::string src = make_source(dim, sigma, load, degree, &nq);
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "fem_rtc.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
        return fail(FEM_ERR_HIP, "hiprtcCreateProgram failed");
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-ffp-contract=on", "-Xclang",
                          "-target-feature", "-Xclang", "-packed-fp32-ops"};
    hiprtcResult rc = hiprtcCompileProgram(prog, 7, opts);
    if (rc != HIPRTC_SUCCESS) {
        size_t n = 0;
        (void)hiprtcGetProgramLogSize(prog, &n);
        std::string log(n + 1, '\0');
        (void)hiprtcGetProgramLog(prog, &log[0]);
        (void)hiprtcDestroyProgram(&prog);
        if (log.size() > 2000) log.resize(2000);
        return fail(FEM_ERR_INVALID_ARG, std::string("integrand does not compile: ") + log.c_str());
    }
    size_t n = 0;
    (void)hiprtcGetCodeSize(prog, &n);
    auto *r = new fem_rtc;
    r->code.resize(n);
    (void)hiprtcGetCode(prog, r->code.data());
    (void)hiprtcDestroyProgram(&prog);
    r->dim = dim;
    r->np = dim + 1;
    r->nq = nq;
    r->has_load = load != nullptr;
    r->source = std::move(src);
    *out = r;
    return FEM_OK;
}

int fem_rtc_source(const fem_rtc *r, char *buf, int64_t size)
{
    clear_error();
    if (!r) return fail(FEM_ERR_INVALID_ARG, "rtc is NULL");
    const int64_t need = (int64_t)r->source.size() + 1;
    if (!buf || size < need) return (int)need;
    std::memcpy(buf, r->source.c_str(), (size_t)need);
    return FEM_OK;
}

int fem_rtc_element_matrices(fem_rtc *r, const fem_mesh *mesh, const double *coef, double reaction,
                             double *elmat, void *stream)
{
    clear_error();
    TraceRange trace_range("fem_rtc_element_matrices");
    if (!r) return fail(FEM_ERR_INVALID_ARG, "rtc is NULL");
    FEM_TRY(check_mesh(mesh, true));
    if (mesh->order != 1 || mesh->dim != r->dim)
        return fail(FEM_ERR_INVALID_ARG, "the mesh does not match the compiled form (P1, its dim)");
    if (mesh->n_elems == 0) return FEM_OK;
    if (!coef || !elmat) return fail(FEM_ERR_INVALID_ARG, "coef or elmat is NULL");
    hipFunction_t fn;
    FEM_TRY(rtc_function(r, &fn));
    const double *coords = mesh->coords;
    const int32_t *conn = mesh->conn;
    long N = (long)mesh->n_nodes, E = (long)mesh->n_elems;
    double c = reaction;
    void *args[] = {&coords, &N, &conn, &E, &coef, &c, &elmat};
    const unsigned blocks = grid_for(E, 256);
    FEM_HIP_TRY(hipModuleLaunchKernel(fn, blocks, 1, 1, 256, 1, 1, 0, (hipStream_t)stream, args,
                                      nullptr));
    return FEM_OK;
}

int fem_assemble_rtc(const fem_pattern *p, const fem_mesh *mesh, fem_rtc *r, const double *coef,
                     double reaction, double *values, double *rhs, unsigned flags, void *stream)
{
    clear_error();
    TraceRange trace_range("fem_assemble_rtc");
    if (!r) return fail(FEM_ERR_INVALID_ARG, "rtc is NULL");
    FEM_TRY(check_mesh(mesh, true));
    FEM_TRY(check_same_mesh(p, mesh));
    if (mesh->order != 1 || mesh->dim != r->dim || p->ncomp != 1)
        return fail(FEM_ERR_INVALID_ARG, "the mesh does not match the compiled form (scalar P1, its dim)");
    hipStream_t s = (hipStream_t)stream;
    const int64_t E = mesh->n_elems;
    const int64_t rows = r->np * r->np + (r->has_load ? r->np : 0);
    double *elmat = nullptr;
    if (E > 0) {
        FEM_HIP_TRY(hipMallocAsync((void **)&elmat, sizeof(double) * (size_t)(rows * E), s));
        int rc = fem_rtc_element_matrices(r, mesh, coef, reaction, elmat, stream);
        if (rc != FEM_OK) {
            (void)hipFreeAsync(elmat, s);
            return rc;
        }
    }
    fem_form f{};
    f.kind = FEM_FORM_ELEMENT_MATRICES;
    f.load = r->has_load ? FEM_LOAD_ELEMENT : FEM_LOAD_NONE;
    int rc = fem_assemble(p, mesh, &f, elmat ? elmat : coef, values, r->has_load ? rhs : nullptr,
                          flags, stream);
    if (elmat) (void)hipFreeAsync(elmat, s);
    return rc;
}

int fem_assemble_backward_rtc(const fem_pattern *p, const fem_mesh *mesh, fem_rtc *r,
                              const double *coef, double reaction, const double *grad_values,
                              const double *grad_rhs, double *grad_coef, double *grad_coords,
                              unsigned flags, void *stream)
{
    clear_error();
    TraceRange trace_range("fem_assemble_backward_rtc");
    (void)coef;
    (void)reaction;
    (void)grad_rhs;  // the load does not depend on kappa
    if (!r) return fail(FEM_ERR_INVALID_ARG, "rtc is NULL");
    FEM_TRY(check_mesh(mesh, true));
    FEM_TRY(check_same_mesh(p, mesh));
    if (mesh->order != 1 || mesh->dim != r->dim || p->ncomp != 1)
        return fail(FEM_ERR_INVALID_ARG, "the mesh does not match the compiled form (scalar P1, its dim)");
    if (grad_coords)
        return fail(FEM_ERR_UNSUPPORTED, "compiled integrands are not differentiated in x");
    if (flags & ~FEM_ACCUMULATE)
        return fail(FEM_ERR_INVALID_ARG, "fem_assemble_backward_rtc takes FEM_ACCUMULATE only");
    const int64_t E = mesh->n_elems;
    if (!grad_coef || E == 0) return FEM_OK;
    hipStream_t s = (hipStream_t)stream;
    if (!grad_values) {
        if (!(flags & FEM_ACCUMULATE)) FEM_TRY(fill_zero_f64(grad_coef, E, s));
        return FEM_OK;
    }
    const int np = r->np;
    const int64_t rows = np * np + (r->has_load ? np : 0);
    double *buf = nullptr;
    FEM_HIP_TRY(hipMallocAsync((void **)&buf, sizeof(double) * (size_t)((rows + 1) * E), s));
    double *ones = buf + rows * E;
    hipLaunchKernelGGL(k_fill_ones, dim3(grid_for(E, 256)), dim3(256), 0, s, ones, E);
    int rc = fem_rtc_element_matrices(r, mesh, ones, 0.0, buf, stream);
    if (rc == FEM_OK)
        hipLaunchKernelGGL(k_rtc_dkappa, dim3(grid_for(E, 256)), dim3(256), 0, s, p->slot, E, np,
                           buf, grad_values, grad_coef, (flags & FEM_ACCUMULATE) != 0);
    (void)hipFreeAsync(buf, s);
    if (rc != FEM_OK) return rc;
    FEM_HIP_TRY(hipGetLastError());
    return FEM_OK;
}

void fem_rtc_destroy(fem_rtc *r)
{
    if (!r) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : r->loaded) {
        (void)hipSetDevice(kv.first);
        (void)hipDeviceSynchronize();
        (void)hipModuleUnload(kv.second.first);
    }
    (void)hipSetDevice(cur);
    delete r;
}

}  // extern "C"
