// P2 tetrahedra, isotropic linear elasticity (the paper's Sec. 7 outlook: higher order):
// a(u, v) = (lam div u, div v) + (2 mu eps(u), eps(v)), three interleaved components per
// node (dof 3n + a), with the 14-point degree-5 rule (exact for this degree-2 integrand).
//
// Local matrix.  With P[q][(i,a)] = sqrt(w_q |T|) d_a phi_i(x_q) (30 columns, padded to
// 32; 14 quadrature rows, padded to 16), the quadrature sum of B^T D B for isotropic D
// splits into the gradient Gram matrix G = P^T P:
//     K[(i,a),(j,b)] = lam G[(i,a),(j,b)] + mu G[(i,b),(j,a)] + mu delta_ab sum_c G[(i,c),(j,c)].
// G is the dense contraction; it runs on the matrix cores: four v_mfma_f64_16x16x4f64
// per 16x16 output tile (K = 16 quadrature rows), one output tile per wavefront, so the
// four wavefronts of a workgroup produce one element's 32x32 G together.  The FP32
// variant rounds P to FP32 and accumulates G in FP32 (v_mfma_f32_16x16x4f32); K and the
// scatter stay FP64.
//
// Scatter.  Same tile scheme as P1: the workgroup's tile of consecutive elements is
// combined in LDS per distinct node pair (a 3x3 block), elements one after the other
// (deterministic), then every distinct pair updates its 9 CSR values once -- device-scope
// atomics, or colour by colour with stores (first writer) and read-modify-writes.  The
// dof-level slot of (3n+a, 3m+b), m at position p of node row n (length L), is
// 9 rowptr[n] + 3 a L + 3 p + b.
#include "fem_internal.h"
#include "quadrature.h"

namespace fem {

namespace {

enum Mode : int { kAtomic = 0, kColoured = 1, kOrdered = 2 };
constexpr int kP2Threads = 256;  // four wavefronts
constexpr int NPE = 10;

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// P2 edge k (local node 4+k) joins vertices (kEdge0[k], kEdge1[k])
__host__ __device__ constexpr int edge_v(int k, int end)
{
    return end == 0 ? (k < 3 ? 0 : (k < 5 ? 1 : 2)) : (k == 0 ? 1 : (k == 1 ? 2 : (k == 2 ? 3 : (k == 3 ? 2 : 3))));
}

// d phi_i / d lambda_v at barycentric point lam (P2 Lagrange basis)
__host__ __device__ constexpr double dphi_dlam(int i, int v, const double *lam)
{
    if (i < 4) return (v == i) ? 4.0 * lam[i] - 1.0 : 0.0;
    const int a = edge_v(i - 4, 0), b = edge_v(i - 4, 1);
    return (v == a) ? 4.0 * lam[b] : ((v == b) ? 4.0 * lam[a] : 0.0);
}

// phi_i at barycentric point lam
__host__ __device__ constexpr double phi(int i, const double *lam)
{
    if (i < 4) return lam[i] * (2.0 * lam[i] - 1.0);
    return 4.0 * lam[edge_v(i - 4, 0)] * lam[edge_v(i - 4, 1)];
}

// reference gradient d phi_i / d xi_m at rule point q (xi_m = lambda_{m+1})
__device__ __forceinline__ double ref_grad(int q, int i, int m)
{
    double lam[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) lam[k] = quad::Tet14::lam(q, k);
    return dphi_dlam(i, m + 1, lam) - dphi_dlam(i, 0, lam);
}

// (1/|T|) int phi_i by the rule (exact: degree 2)
__device__ __forceinline__ double phi_mean(int i)
{
    double s = 0.0;
    for (int q = 0; q < quad::Tet14::nq; ++q) {
        double lam[4];
        for (int k = 0; k < 4; ++k) lam[k] = quad::Tet14::lam(q, k);
        s += quad::Tet14::w(q) * phi(i, lam);
    }
    return s;
}

struct P2Args {
    const double *coords;
    int64_t N, E;
    int T;
    const int32_t *rowptr;  // node level
    const int32_t *tnode_ptr;
    const int32_t *tnode;
    const uint64_t *trun;    // 2 words per tile node
    const uint64_t *tfirst;  // 2 words per tile node
    const uint8_t *trfirst;
    const uint16_t *enode;  // [E][10] tile-node index of each local node
    const uint8_t *epos;    // [E][100] row position of each local pair
    const int32_t *tile_list;
    const int32_t *pred_ptr, *pred;
    int32_t *ctrl;
    int64_t n_tiles;
    const double *lam, *mu;
    int load;
    double bf[3];
    double *values, *rhs;
    int nmax, smax;
    bool use_first;
};

// LDS carve-up
struct P2Lds {
    double *R;      // [14][10][3] reference gradients
    double *G;      // [4][32][32] Gram matrices of the wavefronts' current elements
    double *acc;    // [smax][9] pair accumulators
    double *xs;     // [3][nmax]
    double *racc;   // [3][nmax]
    uint64_t *rb;   // [nmax][2]
    int32_t *ust;   // [nmax]
    int32_t *rp;    // [nmax]
    int32_t *rl;    // [nmax]
    int32_t *nd;    // [nmax]
    int32_t *us;    // [smax]  (first << 31) | (node << 8) | position
    int32_t *scan;  // [16]
    uint16_t *lp;   // [T][100] pair index of (element, i, j)
    uint8_t *nf;    // [nmax]
    __device__ P2Lds(unsigned char *b, int nmax, int smax, int T)
    {
        R = (double *)b;
        G = R + 14 * 10 * 3;
        acc = G + 4 * 32 * 32;
        xs = acc + 9 * smax;
        racc = xs + 3 * nmax;
        rb = (uint64_t *)(racc + 3 * nmax);
        ust = (int32_t *)(rb + 2 * nmax);
        rp = ust + nmax;
        rl = rp + nmax;
        nd = rl + nmax;
        us = nd + nmax;
        scan = us + smax;
        lp = (uint16_t *)(scan + 16);
        nf = (uint8_t *)(lp + T * 100);
    }
};

size_t p2_lds_bytes(int nmax, int smax, int T)
{
    return sizeof(double) * (size_t)(420 + 4 * 1024 + 9 * smax + 6 * nmax) + sizeof(uint64_t) * 2 * nmax +
           sizeof(int32_t) * (size_t)(4 * nmax + smax + 16) + sizeof(uint16_t) * 100 * T + nmax + 16;
}

__device__ int wg_scan_excl(int v, int *sh, int *total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh[w] = x;
    __syncthreads();
    int base = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
        int t = sh[i];
        base += (i < w) ? t : 0;
        tot += t;
    }
    *total = tot;
    __syncthreads();
    return base + x - v;
}

__device__ __forceinline__ int popc_below(const uint64_t *m, int p)
{
    // set bits of the 128-bit mask m[0..1] below position p
    if (p < 64) return __popcll(m[0] & ((1ull << p) - 1ull));
    return __popcll(m[0]) + __popcll(m[1] & ((1ull << (p - 64)) - 1ull));
}

// Affine geometry of the element's 4 vertices: J^{-1} (inv[m][a] = d xi_m / d x_a), |T|
__device__ __forceinline__ void p2_geometry(const double x[4][3], double inv[3][3], double &vol)
{
    double J[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int m = 0; m < 3; ++m) J[a][m] = x[m + 1][a] - x[0][a];
    const double C00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double C01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double C02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * C00 + J[0][1] * C01 + J[0][2] * C02;
    const double r = 1.0 / det;
    inv[0][0] = C00 * r;
    inv[1][0] = C01 * r;
    inv[2][0] = C02 * r;
    inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * r;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * r;
    inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * r;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * r;
    inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * r;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * r;
    vol = fabs(det) * (1.0 / 6.0);
}

// sqrt(w_q) d_a phi_i (x_q) for column c = 3i + a (0 beyond 30 columns / 14 points); the
// table R holds sqrt(w_q) times the reference gradients
__device__ __forceinline__ double pval(const double *R, int q, int c, const double inv[3][3])
{
    if (q >= 14 || c >= 30) return 0.0;
    const int i = c / 3, a = c - 3 * (c / 3);
    const double *r = R + (q * 10 + i) * 3;
    return r[0] * inv[0][a] + r[1] * inv[1][a] + r[2] * inv[2][a];
}

template <int MODE, bool F32>
__global__ __launch_bounds__(kP2Threads) void k_p2_tile_fwd(P2Args a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    P2Lds L(smem, a.nmax, a.smax, a.T);
    __shared__ int s_ticket;
    const int tid = threadIdx.x;
    int64_t tile;
    if (MODE == kOrdered) tile = a.tile_list[take_ticket(a.ctrl, a.n_tiles, &s_ticket)];
    else if (MODE == kColoured) tile = a.tile_list[blockIdx.x];
    else tile = xcd_block(blockIdx.x, gridDim.x);
    const int n0 = a.tnode_ptr[tile];
    const int nn = a.tnode_ptr[tile + 1] - n0;
    const int64_t e0 = tile * a.T;
    const int ne = (int)min((int64_t)a.T, a.E - e0);

    // ---- stage: reference gradients (scaled by sqrt(w_q)), tile nodes, distinct pairs ----
    for (int t = tid; t < 14 * 10 * 3; t += kP2Threads) {
        const int q = t / 30, i = (t / 3) % 10, m = t % 3;
        L.R[t] = sqrt(quad::Tet14::w(q)) * ref_grad(q, i, m);
    }
    const int per = (nn + kP2Threads - 1) / kP2Threads;
    const int k0 = min(nn, tid * per), k1 = min(nn, k0 + per);
    int local = 0;
    for (int k = k0; k < k1; ++k) {
        const int32_t n = a.tnode[n0 + k];
        L.nd[k] = n;
        L.rb[2 * k] = a.trun[2 * (int64_t)(n0 + k)];
        L.rb[2 * k + 1] = a.trun[2 * (int64_t)(n0 + k) + 1];
        L.rp[k] = a.rowptr[n];
        L.rl[k] = a.rowptr[n + 1] - a.rowptr[n];
        L.nf[k] = a.use_first ? a.trfirst[n0 + k] : 0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            L.xs[d * a.nmax + k] = a.coords[d * a.N + n];
            L.racc[d * a.nmax + k] = 0.0;
        }
        local += __popcll(L.rb[2 * k]) + __popcll(L.rb[2 * k + 1]);
    }
    int total = 0;
    int off = wg_scan_excl(local, L.scan, &total);
    for (int k = k0; k < k1; ++k) {
        L.ust[k] = off;
        for (int w = 0; w < 2; ++w) {
            uint64_t r = L.rb[2 * k + w];
            const uint64_t f = a.use_first ? a.tfirst[2 * (int64_t)(n0 + k) + w] : 0ull;
            while (r) {
                const int b = __builtin_ctzll(r);
                L.us[off] = (((f >> b) & 1ull) ? (int32_t)0x80000000 : 0) | (k << 8) | (64 * w + b);
#pragma unroll
                for (int v = 0; v < 9; ++v) L.acc[9 * off + v] = 0.0;
                ++off;
                r &= r - 1;
            }
        }
    }
    __syncthreads();
    for (int t = tid; t < ne * 100; t += kP2Threads) {
        const int el = t / 100, ij = t - 100 * el, i = ij / 10;
        const int64_t e = e0 + el;
        const int ki = a.enode[e * NPE + i];
        const int p = a.epos[e * NPE * NPE + ij];
        L.lp[el * 100 + ij] = (uint16_t)(L.ust[ki] + popc_below(&L.rb[2 * ki], p));
    }
    __syncthreads();

    // ---- elements: one per wavefront, four in flight ----
    const int wave = tid >> 6, lane = tid & 63;
    double *G = L.G + wave * 32 * 32;
    for (int base = 0; base < ne; base += 4) {
        const int el = base + wave;
        const bool has = el < ne;
        double lm = 0.0, mm = 0.0, vol = 0.0;
        if (has) {
            const int64_t e = e0 + el;
            double x[4][3];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int kv = a.enode[e * NPE + v];
#pragma unroll
                for (int d = 0; d < 3; ++d) x[v][d] = L.xs[d * a.nmax + kv];
            }
            double inv[3][3];
            p2_geometry(x, inv, vol);
            const double sv = sqrt(vol);
            lm = a.lam[e];
            mm = a.mu[e];
            // G = P^T P, symmetric: output tiles (0,0), (0,1), (1,1); (1,0) by transposition
            const int lo = lane & 15, hi = lane >> 4;
#pragma unroll
            for (int tb = 0; tb < 3; ++tb) {
                const int rb = tb == 2 ? 1 : 0, cb = tb == 0 ? 0 : 1;
                const int rc = rb * 16 + lo, cc = cb * 16 + lo;
                if constexpr (F32) {
                    f4_t g = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks) {
                        const int q = 4 * ks + hi;
                        const float av = (float)(sv * pval(L.R, q, rc, inv));
                        const float bv = (float)(sv * pval(L.R, q, cc, inv));
                        g = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, g, 0, 0, 0);
                    }
                    // f32 16x16x4 output layout: register r of lane l holds row 4 (l / 16) + r
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int R = rb * 16 + 4 * hi + r, C = cb * 16 + lo;
                        G[R * 32 + C] = (double)g[r];
                        if (tb == 1) G[C * 32 + R] = (double)g[r];
                    }
                } else {
                    d4_t g = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks) {
                        const int q = 4 * ks + hi;
                        const double av = sv * pval(L.R, q, rc, inv);
                        const double bv = sv * pval(L.R, q, cc, inv);
                        g = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, g, 0, 0, 0);
                    }
                    // f64 16x16x4 output layout (measured on gfx950): register r of lane l
                    // holds row (l / 16) + 4 r, column l % 16
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int R = rb * 16 + hi + 4 * r, C = cb * 16 + lo;
                        G[R * 32 + C] = g[r];
                        if (tb == 1) G[C * 32 + R] = g[r];
                    }
                }
            }
        }
        // the Gram matrix was written by other lanes of this wavefront
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // K blocks of this wavefront's element: lanes take node pairs (i, j)
        double kb[2][9];
        int lpi[2] = {0, 0};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int pr = lane + 64 * h;
            if (has && pr < 100) {
                const int i = pr / 10, j = pr - 10 * (pr / 10);
                double gb[3][3];
#pragma unroll
                for (int p = 0; p < 3; ++p)
#pragma unroll
                    for (int q = 0; q < 3; ++q) gb[p][q] = G[(3 * i + p) * 32 + 3 * j + q];
                const double tr = gb[0][0] + gb[1][1] + gb[2][2];
#pragma unroll
                for (int p = 0; p < 3; ++p)
#pragma unroll
                    for (int q = 0; q < 3; ++q)
                        kb[h][3 * p + q] = lm * gb[p][q] + mm * gb[q][p] + (p == q ? mm * tr : 0.0);
                lpi[h] = L.lp[el * 100 + pr];
            }
        }
        // all reads of G done before the next element overwrites it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double bfv[3] = {0.0, 0.0, 0.0};
        int bnode = 0;
        if (a.load == FEM_LOAD_CONST && has && lane < 10) {
            // body force: b[(i,c)] = f_c |T| (1/|T|) int phi_i
            bnode = a.enode[(e0 + el) * NPE + lane];
            const double pm = phi_mean(lane);
#pragma unroll
            for (int c = 0; c < 3; ++c) bfv[c] = a.bf[c] * vol * pm;
        }
        if (MODE == kAtomic) {
#pragma unroll
            for (int h = 0; h < 2; ++h)
                if (has && lane + 64 * h < 100)
#pragma unroll
                    for (int v = 0; v < 9; ++v) atomicAdd(&L.acc[9 * lpi[h] + v], kb[h][v]);
            if (a.load == FEM_LOAD_CONST && has && lane < 10)
#pragma unroll
                for (int c = 0; c < 3; ++c) atomicAdd(&L.racc[c * a.nmax + bnode], bfv[c]);
        } else {
            // deterministic: the four elements are added in element order
            for (int w2 = 0; w2 < 4; ++w2) {
                if (wave == w2) {
#pragma unroll
                    for (int h = 0; h < 2; ++h)
                        if (has && lane + 64 * h < 100)
#pragma unroll
                            for (int v = 0; v < 9; ++v) L.acc[9 * lpi[h] + v] += kb[h][v];
                    if (a.load == FEM_LOAD_CONST && has && lane < 10)
#pragma unroll
                        for (int c = 0; c < 3; ++c) L.racc[c * a.nmax + bnode] += bfv[c];
                }
                __syncthreads();
            }
        }
    }
    __syncthreads();

    // ---- one global update per distinct (pair, a, b) and per (node, a) ----
    const int nvals = 9 * total;
    if (MODE == kOrdered) {
        wait_preds(a.pred_ptr, a.pred, a.ctrl, a.n_tiles, tile);
        auto slot_of = [&](int t) {
            const int ra = t / (3 * total), rest = t - ra * 3 * total;
            const int u = rest / 3, cb = rest - 3 * (rest / 3);
            const int32_t code = L.us[u];
            const int k = (code >> 8) & 0xffff, p = code & 0xff;
            return 9 * (int64_t)L.rp[k] + 3 * (int64_t)ra * L.rl[k] + 3 * p + cb;
        };
        auto val_of = [&](int t) {
            const int ra = t / (3 * total), rest = t - ra * 3 * total;
            const int u = rest / 3, cb = rest - 3 * (rest / 3);
            return L.acc[9 * u + 3 * ra + cb];
        };
        auto first_of = [&](int t) { return L.us[(t - (t / (3 * total)) * 3 * total) / 3] < 0; };
        ordered_rmw<8>(a.values, nvals, slot_of, val_of, first_of);
        if (a.load == FEM_LOAD_CONST)
            ordered_rmw<4>(
                a.rhs, 3 * nn, [&](int t) { return 3 * (int64_t)L.nd[t / 3] + t % 3; },
                [&](int t) { return L.racc[(t % 3) * a.nmax + t / 3]; },
                [&](int t) { return L.nf[t / 3] != 0; });
        publish_done(a.ctrl, tile);
        return;
    }
    for (int t = tid; t < nvals; t += kP2Threads) {
        const int ra = t / (3 * total), rest = t - ra * 3 * total;
        const int u = rest / 3, cb = rest - 3 * (rest / 3);
        const int32_t code = L.us[u];
        const int k = (code >> 8) & 0xffff, p = code & 0xff;
        const int64_t slot = 9 * (int64_t)L.rp[k] + 3 * (int64_t)ra * L.rl[k] + 3 * p + cb;
        const double v = L.acc[9 * u + 3 * ra + cb];
        if (MODE == kAtomic) unsafeAtomicAdd(a.values + slot, v);
        else if (code < 0) a.values[slot] = v;
        else a.values[slot] += v;
    }
    if (a.load == FEM_LOAD_CONST) {
        for (int t = tid; t < 3 * nn; t += kP2Threads) {
            const int k = t / 3, c = t - 3 * (t / 3);
            double *dst = a.rhs + 3 * (int64_t)L.nd[k] + c;
            const double v = L.racc[c * a.nmax + k];
            if (MODE == kAtomic) unsafeAtomicAdd(dst, v);
            else if (L.nf[k]) *dst = v;
            else *dst += v;
        }
    }
}

template <class K>
void p2_launch(K kernel, const fem_pattern *p, P2Args a, int mode, size_t lds, hipStream_t s)
{
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
    if (mode == kAtomic) {
        a.tile_list = nullptr;
        hipLaunchKernelGGL(kernel, dim3((unsigned)p->n_tiles), dim3(kP2Threads), lds, s, a);
        return;
    }
    if (mode == kOrdered) {
        a.tile_list = p->tile_perm;
        (void)fill_zero_i32(p->tctrl, p->n_tiles + 2, s);
        hipLaunchKernelGGL(kernel, dim3((unsigned)p->n_tiles), dim3(kP2Threads), lds, s, a);
        return;
    }
    for (int c = 0; c < p->n_tile_colours; ++c) {
        int64_t b = p->tile_colour_ptr[c], n = p->tile_colour_ptr[c + 1] - b;
        if (n <= 0) continue;
        a.tile_list = p->tile_perm + b;
        hipLaunchKernelGGL(kernel, dim3((unsigned)n), dim3(kP2Threads), lds, s, a);
    }
}

}  // namespace

int p2_tile_forward(const fem_pattern *p, const fem_mesh *m, const fem_form *f, const double *coef,
                    double *values, double *rhs, unsigned flags, hipStream_t s)
{
    if (p->n_tiles == 0) return FEM_OK;
    const int mode = !(flags & FEM_SCATTER_COLOURED) ? kAtomic
                     : ((flags & FEM_COLOUR_LAUNCHES) ? kColoured : kOrdered);
    P2Args a{};
    a.coords = m->coords;
    a.N = m->n_nodes;
    a.E = m->n_elems;
    a.T = p->tile;
    a.rowptr = p->rowptr_n;
    a.tnode_ptr = p->tnode_ptr;
    a.tnode = p->tnode;
    a.trun = p->trun;
    a.tfirst = p->tfirst;
    a.trfirst = p->trfirst;
    a.enode = p->enode16;
    a.epos = p->epos8;
    a.pred_ptr = p->tpred_ptr;
    a.pred = p->tpred;
    a.ctrl = p->tctrl;
    a.n_tiles = p->n_tiles;
    a.lam = coef;
    a.mu = coef + m->n_elems;
    a.load = rhs ? f->load : FEM_LOAD_NONE;
    for (int c = 0; c < 3; ++c) a.bf[c] = f->load_const[c];
    a.values = values;
    a.rhs = rhs;
    a.nmax = p->tile_max_nodes;
    a.smax = p->tile_max_slots;
    a.use_first = mode != kAtomic && !(flags & FEM_ACCUMULATE);
    if (a.T > 64) return fail(FEM_ERR_UNSUPPORTED, "P2 tiles hold at most 64 elements");
    const size_t lds = p2_lds_bytes(a.nmax, a.smax, a.T);
    if (lds > 160 * 1024) return fail(FEM_ERR_UNSUPPORTED, "P2 tile needs more LDS than a CU has");
    const bool f32 = (flags & FEM_PREC_FP32) != 0;
    if (mode == kOrdered) {
        if (f32) p2_launch(k_p2_tile_fwd<kOrdered, true>, p, a, mode, lds, s);
        else p2_launch(k_p2_tile_fwd<kOrdered, false>, p, a, mode, lds, s);
    } else if (mode == kColoured) {
        if (f32) p2_launch(k_p2_tile_fwd<kColoured, true>, p, a, mode, lds, s);
        else p2_launch(k_p2_tile_fwd<kColoured, false>, p, a, mode, lds, s);
    } else {
        if (f32) p2_launch(k_p2_tile_fwd<kAtomic, true>, p, a, mode, lds, s);
        else p2_launch(k_p2_tile_fwd<kAtomic, false>, p, a, mode, lds, s);
    }
    FEM_HIP_TRY(hipGetLastError());
    return FEM_OK;
}

int p2_tile_backward(const fem_pattern *, const fem_mesh *, const fem_form *, const double *,
                     const double *, const double *, double *, double *, unsigned, hipStream_t)
{
    return fail(FEM_ERR_UNSUPPORTED, "elasticity adjoint not available in this build");
}

}  // namespace fem
