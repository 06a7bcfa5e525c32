// P1 scalar assembly, -div(kappa sigma grad u) + c u = f (Sec. 4.1, Eq. (1)-(3); sigma = I
// or an affine matrix field), and its adjoint, on triangles (D = 2) and tetrahedra
// (D = 3), one element per thread with no tile combining.
//
// One thread per element (Alg. 1 gives each element a block of threads, one per
// quadrature point and local entry; on CDNA a 4x4 P1 element is too little work to split
// over 64 lanes, so a lane owns an element and the quadrature loop runs in registers).
// Per element:
//   geometry    J[a][m] = x_{m+1,a} - x_{0,a},  det J,  J^{-1} by cofactors,
//               vol = |det J| / D!
//   gradients   B = Ghat J^{-1} (row i = grad lambda_i; Ghat rows: (-1,..,-1), e_1..e_D)
//   stiffness   kappa vol B S B^T (S = I, or sigma at the centroid: the integrand is
//               affine on an affine element, so one evaluation is its exact integral)
//   mass        c vol M, M_ij = sum_q w_q lam_i(q) lam_j(q)    (folded at compile time)
//   load        b_i = vol sum_q w_q f(x_q) lam_i(q),  x_q = sum_k lam_k(q) x_k
//   (the arithmetic is p1_element.h's, shared with the tile kernels)
//   scatter     values[slot(e,i,j)] += A_ij, rhs[conn_i] += b_i  (Alg. 1, last step):
//               device-scope FP64 atomics, or plain read-modify-write when the launch
//               covers one colour (no two elements of a colour share a node).
#include "fem_internal.h"
#include "p1_element.h"
#include "quadrature.h"

namespace fem {

namespace {

constexpr int kThreads = 256;

enum Mode : int { kAtomic = 0, kColoured = 1 };

struct P1Args {
    const double *coords;  // [D][N]
    int64_t N;
    const int32_t *conn;  // [D+1][E] (colour order when coloured)
    const int32_t *slot;  // [(D+1)^2][E]
    const int32_t *perm;  // element id of each position (coloured) or null
    int64_t E;            // stride of conn/slot
    int64_t begin, count; // positions [begin, begin+count)
    const double *kappa;
    P1Form form;
    double *values, *rhs;
    int *err;
    bool accumulate_unused;
};

__device__ __forceinline__ void scatter_add(double *p, double v, int mode)
{
    if (mode == kAtomic) unsafeAtomicAdd(p, v);
    else *p += v;
}

template <int D, int LOAD, int MODE, int FORM>
__global__ __launch_bounds__(kThreads) void k_p1_fwd(P1Args a)
{
    constexpr int NP = D + 1;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t t = blk * kThreads + threadIdx.x;
    if (t >= a.count) return;
    const int64_t pos = a.begin + t;
    const int64_t e = (MODE == kColoured) ? (int64_t)a.perm[pos] : pos;

    Elem<D> g;
    int32_t v[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) v[k] = a.conn[k * a.E + pos];
#pragma unroll
    for (int k = 0; k < NP; ++k)
#pragma unroll
        for (int d = 0; d < D; ++d) g.x[k][d] = a.coords[d * a.N + v[k]];
    double A[NP][NP], b[NP];
    if constexpr (FORM == FEM_FORM_ELEMENT_MATRICES) p1_given<D, LOAD>(a.kappa, a.E, e, A, b);
    else p1_local<D, FORM, LOAD>(a.form, g, a.kappa[e], A, b);
    if (FORM != FEM_FORM_ELEMENT_MATRICES && a.err && g.det == 0.0) atomicOr(a.err, 1);
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            int32_t s = a.slot[(int64_t)(i * NP + j) * a.E + pos];
            scatter_add(a.values + s, A[i][j], MODE);
        }
    if constexpr (LOAD != FEM_LOAD_NONE) {
#pragma unroll
        for (int i = 0; i < NP; ++i) scatter_add(a.rhs + v[i], b[i], MODE);
    }
}

// ---- adjoint (formulas in p1_element.h) ---------------------------------------------
struct P1BwdArgs {
    P1Args f;
    const double *gvalues, *grhs;
    double *gkappa, *gcoords;
    bool accumulate;
};

template <int D, int LOAD, int MODE, int FORM>
__global__ __launch_bounds__(kThreads) void k_p1_bwd(P1BwdArgs b)
{
    constexpr int NP = D + 1;
    const P1Args &a = b.f;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t t = blk * kThreads + threadIdx.x;
    if (t >= a.count) return;
    const int64_t pos = a.begin + t;
    const int64_t e = (MODE == kColoured) ? (int64_t)a.perm[pos] : pos;

    Elem<D> g;
    int32_t v[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) v[k] = a.conn[k * a.E + pos];
#pragma unroll
    for (int k = 0; k < NP; ++k)
#pragma unroll
        for (int d = 0; d < D; ++d) g.x[k][d] = a.coords[d * a.N + v[k]];
    elem_geometry<D>(g);

    double G[NP][NP];
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
        for (int j = 0; j < NP; ++j)
            G[i][j] = b.gvalues ? b.gvalues[a.slot[(int64_t)(i * NP + j) * a.E + pos]] : 0.0;
    double S[D][D], M[D][D], s, msum;
    p1_adj_scalars<D, FORM>(a.form, g, G, S, M, s, msum);
    if (b.gkappa) {
        double dk = g.vol * s;
        if (b.accumulate) b.gkappa[e] += dk;
        else b.gkappa[e] = dk;
    }
    if (!b.gcoords) return;

    double gb[NP], xbar[NP][D];
#pragma unroll
    for (int i = 0; i < NP; ++i) gb[i] = (LOAD != FEM_LOAD_NONE && b.grhs) ? b.grhs[v[i]] : 0.0;
    p1_adj_coords<D, FORM, LOAD>(a.form, g, a.kappa[e], G, S, M, gb, s, msum, xbar);
#pragma unroll
    for (int k = 0; k < NP; ++k)
#pragma unroll
        for (int d = 0; d < D; ++d) scatter_add(b.gcoords + d * a.N + v[k], xbar[k][d], MODE);
}

template <int D, int LOAD, int MODE, int FORM>
void launch_fwd(const P1Args &a, hipStream_t s)
{
    if (a.count <= 0) return;
    hipLaunchKernelGGL((k_p1_fwd<D, LOAD, MODE, FORM>), dim3(grid_for(a.count, kThreads)), dim3(kThreads),
                       0, s, a);
}

template <int D, int LOAD, int MODE, int FORM>
void launch_bwd(const P1BwdArgs &b, hipStream_t s)
{
    if (b.f.count <= 0) return;
    hipLaunchKernelGGL((k_p1_bwd<D, LOAD, MODE, FORM>), dim3(grid_for(b.f.count, kThreads)),
                       dim3(kThreads), 0, s, b);
}

template <int D, int LOAD, int FORM>
void run_fwd(const fem_pattern *p, P1Args a, bool coloured, hipStream_t s)
{
    if (!coloured) {
        a.conn = a.conn;  // caller's connectivity, element order
        a.slot = p->slot;
        a.perm = nullptr;
        a.begin = 0;
        a.count = p->n_elems;
        launch_fwd<D, LOAD, kAtomic, FORM>(a, s);
        return;
    }
    a.conn = p->conn_perm;
    a.slot = p->slot_perm;
    a.perm = p->perm;
    for (int c = 0; c < p->n_colours; ++c) {
        a.begin = p->colour_ptr[c];
        a.count = p->colour_ptr[c + 1] - p->colour_ptr[c];
        launch_fwd<D, LOAD, kColoured, FORM>(a, s);
    }
}

template <int D, int LOAD, int FORM>
void run_bwd(const fem_pattern *p, P1BwdArgs b, bool coloured, hipStream_t s)
{
    if (!coloured) {
        b.f.slot = p->slot;
        b.f.perm = nullptr;
        b.f.begin = 0;
        b.f.count = p->n_elems;
        launch_bwd<D, LOAD, kAtomic, FORM>(b, s);
        return;
    }
    b.f.conn = p->conn_perm;
    b.f.slot = p->slot_perm;
    b.f.perm = p->perm;
    for (int c = 0; c < p->n_colours; ++c) {
        b.f.begin = p->colour_ptr[c];
        b.f.count = p->colour_ptr[c + 1] - p->colour_ptr[c];
        launch_bwd<D, LOAD, kColoured, FORM>(b, s);
    }
}

template <int D, int FORM>
void dispatch_fwd_load(const fem_pattern *p, const P1Args &a, int load, bool coloured, hipStream_t s)
{
    switch (load) {
    case FEM_LOAD_NONE: run_fwd<D, FEM_LOAD_NONE, FORM>(p, a, coloured, s); break;
    case FEM_LOAD_CONST: run_fwd<D, FEM_LOAD_CONST, FORM>(p, a, coloured, s); break;
    case FEM_LOAD_POLY2: run_fwd<D, FEM_LOAD_POLY2, FORM>(p, a, coloured, s); break;
    default: run_fwd<D, FEM_LOAD_SINPROD, FORM>(p, a, coloured, s); break;
    }
}

template <int D, int FORM>
void dispatch_bwd_load(const fem_pattern *p, const P1BwdArgs &b, int load, bool coloured, hipStream_t s)
{
    switch (load) {
    case FEM_LOAD_NONE: run_bwd<D, FEM_LOAD_NONE, FORM>(p, b, coloured, s); break;
    case FEM_LOAD_CONST: run_bwd<D, FEM_LOAD_CONST, FORM>(p, b, coloured, s); break;
    case FEM_LOAD_POLY2: run_bwd<D, FEM_LOAD_POLY2, FORM>(p, b, coloured, s); break;
    default: run_bwd<D, FEM_LOAD_SINPROD, FORM>(p, b, coloured, s); break;
    }
}

template <int D>
void dispatch_fwd(const fem_pattern *p, const P1Args &a, int form, int load, bool coloured,
                  hipStream_t s)
{
    if (form == FEM_FORM_ELEMENT_MATRICES) {
        if (load == FEM_LOAD_ELEMENT)
            run_fwd<D, FEM_LOAD_ELEMENT, FEM_FORM_ELEMENT_MATRICES>(p, a, coloured, s);
        else run_fwd<D, FEM_LOAD_NONE, FEM_FORM_ELEMENT_MATRICES>(p, a, coloured, s);
        return;
    }
    if (form == FEM_FORM_HELMHOLTZ_SIGMA)
        dispatch_fwd_load<D, FEM_FORM_HELMHOLTZ_SIGMA>(p, a, load, coloured, s);
    else dispatch_fwd_load<D, FEM_FORM_HELMHOLTZ>(p, a, load, coloured, s);
}

template <int D>
void dispatch_bwd(const fem_pattern *p, const P1BwdArgs &b, int form, int load, bool coloured,
                  hipStream_t s)
{
    if (form == FEM_FORM_HELMHOLTZ_SIGMA)
        dispatch_bwd_load<D, FEM_FORM_HELMHOLTZ_SIGMA>(p, b, load, coloured, s);
    else dispatch_bwd_load<D, FEM_FORM_HELMHOLTZ>(p, b, load, coloured, s);
}

__global__ void k_p1_validate(const double *__restrict__ coords, int64_t N,
                              const int32_t *__restrict__ conn, int64_t E, int D, int *err)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    double x[4][3] = {};
    for (int k = 0; k <= D; ++k)
        for (int d = 0; d < D; ++d) x[k][d] = coords[d * N + conn[k * E + e]];
    double det;
    if (D == 2) {
        det = (x[1][0] - x[0][0]) * (x[2][1] - x[0][1]) - (x[2][0] - x[0][0]) * (x[1][1] - x[0][1]);
    } else {
        double a[3][3];
        for (int d = 0; d < 3; ++d)
            for (int m = 0; m < 3; ++m) a[d][m] = x[m + 1][d] - x[0][d];
        det = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
              a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
              a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
    }
    if (!(det != 0.0) || !isfinite(det)) atomicOr(err, 1);
}

}  // namespace

// Device-side check that no element has a zero (or non-finite) Jacobian determinant.
// Reads the vertex coordinates only; synchronises the stream.
int validate_elements(const fem_mesh *m, hipStream_t s)
{
    if (m->n_elems == 0) return FEM_OK;
    int *d_err = nullptr;
    FEM_HIP_TRY(hipMallocAsync((void **)&d_err, sizeof(int), s));
    FEM_HIP_TRY(hipMemsetAsync(d_err, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_p1_validate, dim3(grid_for(m->n_elems, kThreads)), dim3(kThreads), 0, s,
                       m->coords, m->n_nodes, m->conn, m->n_elems, (int)m->dim, d_err);
    int h = 0;
    FEM_HIP_TRY(hipMemcpyAsync(&h, d_err, sizeof(int), hipMemcpyDeviceToHost, s));
    FEM_HIP_TRY(hipStreamSynchronize(s));
    (void)hipFreeAsync(d_err, s);
    if (h) return fail(FEM_ERR_DEGENERATE, "element with zero Jacobian determinant");
    return FEM_OK;
}

int p1_forward(const fem_pattern *p, const fem_mesh *m, const fem_form *f, const double *coef,
               double *values, double *rhs, unsigned flags, hipStream_t s)
{
    P1Args a{};
    a.coords = m->coords;
    a.N = m->n_nodes;
    a.conn = m->conn;
    a.E = m->n_elems;
    a.kappa = coef;
    a.form = p1_form_of(f);
    a.values = values;
    a.rhs = rhs;
    int *d_err = nullptr;
    if (flags & FEM_VALIDATE) {
        FEM_HIP_TRY(hipMallocAsync((void **)&d_err, sizeof(int), s));
        FEM_HIP_TRY(hipMemsetAsync(d_err, 0, sizeof(int), s));
    }
    a.err = d_err;
    bool coloured = (flags & FEM_SCATTER_COLOURED) != 0;
    int load = rhs ? f->load : FEM_LOAD_NONE;
    if (m->dim == 2) dispatch_fwd<2>(p, a, f->kind, load, coloured, s);
    else dispatch_fwd<3>(p, a, f->kind, load, coloured, s);
    FEM_HIP_TRY(hipGetLastError());
    if (d_err) {
        int h = 0;
        FEM_HIP_TRY(hipMemcpyAsync(&h, d_err, sizeof(int), hipMemcpyDeviceToHost, s));
        FEM_HIP_TRY(hipStreamSynchronize(s));
        (void)hipFreeAsync(d_err, s);
        if (h) return fail(FEM_ERR_DEGENERATE, "element with zero Jacobian determinant");
    }
    return FEM_OK;
}

int p1_backward(const fem_pattern *p, const fem_mesh *m, const fem_form *f, const double *coef,
                const double *gvalues, const double *grhs, double *gcoef, double *gcoords,
                unsigned flags, hipStream_t s)
{
    P1BwdArgs b{};
    b.f.coords = m->coords;
    b.f.N = m->n_nodes;
    b.f.conn = m->conn;
    b.f.E = m->n_elems;
    b.f.kappa = coef;
    b.f.form = p1_form_of(f);
    b.gvalues = gvalues;
    b.grhs = grhs;
    b.gkappa = gcoef;
    b.gcoords = gcoords;
    b.accumulate = (flags & FEM_ACCUMULATE) != 0;
    bool coloured = (flags & FEM_SCATTER_COLOURED) != 0;
    int load = grhs ? f->load : FEM_LOAD_NONE;
    if (m->dim == 2) dispatch_bwd<2>(p, b, f->kind, load, coloured, s);
    else dispatch_bwd<3>(p, b, f->kind, load, coloured, s);
    FEM_HIP_TRY(hipGetLastError());
    return FEM_OK;
}

}  // namespace fem
