// multigrid.hip -- CG preconditioned by a multigrid V-cycle for the
// finite-volume Poisson operator of Eq. poi.
//
// Hierarchy: each coarse node aggregates the (up to) 2x2x2 nodes below it;
// the prolongation P is piecewise constant and the coarse operator is the
// Galerkin product P^T A P, which stays a 7-point stencil on the structured
// grid (aggregates couple only through shared faces). Nodes held at a fixed
// potential are not unknowns and belong to no aggregate. The finest level
// uses the operator matrix-free from the node types; coarser levels store
// diag and the +x/+y/+z couplings per node. Smoother: damped Jacobi, the same
// number of sweeps before and after the coarse correction, so the V-cycle is
// a symmetric positive definite preconditioner for CG. The coarsest level
// (at most 1024 nodes) is solved exactly with its inverse, formed once on the
// host at set-up. The finest level runs as z-marching kernels.
#include <cmath>
#include <vector>

#include "pic_internal.hpp"

namespace pic {

constexpr int kMgMaxLevels = 12;

// Storage of every multigrid vector and coarse operator: FP32 (the V-cycle is
// a preconditioner, so its precision decides only how good the search
// directions are; the Krylov vectors, dot products and the convergence test
// stay FP64). Arithmetic inside the kernels is FP64.
typedef float mgv;
constexpr int kMgBlocks = 1024;
constexpr double kOmega = 6.0 / 7.0;  // damped Jacobi weight for 7-point stencils

struct MgLevel {
    int nx, ny, nz;
    int64_t n;
    mgv *diag, *cx, *cy, *cz;  // levels >= 1
    mgv *x0, *x1, *b;          // x ping-pong and right-hand side (b: levels >= 1)
};

struct MgHier {
    int nlev;
    MgLevel lv[kMgMaxLevels];
    mgv* z[2];     // finest-level preconditioned residual (ping-pong)
    double* part;  // partial sums
    double* cinv;  // inverse of the coarsest operator, n x n (zero rows / columns for fixed nodes)
    int pre, post;
    double alpha_c;
    int zm_kc, zr_kc;          // planes per block of the fine sweeps / the fine restriction
    unsigned zm_blocks, zr_blocks;
};

static void mg_dims(const pic_config* cfg, std::vector<int3>& dims) {
    int nx = cfg->nx, ny = cfg->ny, nz = cfg->nz;
    dims.push_back(make_int3(nx, ny, nz));
    while ((int)dims.size() < kMgMaxLevels) {
        int3 d = dims.back();
        if ((int64_t)d.x * d.y * d.z <= 512 || d.x <= 2 || d.y <= 2 || d.z <= 2) break;
        dims.push_back(make_int3((d.x + 1) / 2, (d.y + 1) / 2, (d.z + 1) / 2));
    }
}

size_t mg_bytes(const pic_config* cfg) {
    std::vector<int3> dims;
    mg_dims(cfg, dims);
    size_t b = 4096 + sizeof(MgHier);
    int64_t nn = (int64_t)cfg->nx * cfg->ny * cfg->nz;
    b += 2 * nn * sizeof(mgv) + 2 * 256 + 64 * kMgBlocks * 8;
    for (size_t l = 1; l < dims.size(); ++l) {
        int64_t n = (int64_t)dims[l].x * dims[l].y * dims[l].z;
        b += 7 * (size_t)n * sizeof(mgv) + 7 * 256;
    }
    int64_t nc = (int64_t)dims.back().x * dims.back().y * dims.back().z;
    if (nc <= 1024) b += (size_t)nc * nc * 8 + 256;
    return b;
}

__device__ inline double hedge(int i, int n) { return (i == 0 || i == n - 1) ? 0.5 : 1.0; }

// ---------------------------------------------------------------------------
// Setup: coarse stencils

// Level 1 from the matrix-free finest operator.
__global__ void k_mg_build1(Grid g, const uint8_t* __restrict__ type, MgLevel c) {
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= c.n) return;
    int Ix = (int)(I % c.nx), Iy = (int)((I / c.nx) % c.ny), Iz = (int)(I / ((int64_t)c.nx * c.ny));
    double dg = 0.0, cx = 0.0, cy = 0.0, cz = 0.0;
    for (int t = 0; t < 8; ++t) {
        int i = 2 * Ix + (t & 1), j = 2 * Iy + ((t >> 1) & 1), k = 2 * Iz + ((t >> 2) & 1);
        if (i >= g.nx || j >= g.ny || k >= g.nz) continue;
        int64_t n = ((int64_t)k * g.ny + j) * g.nx + i;
        if (type[n] != 0) continue;
        double fx = hedge(j, g.ny) * hedge(k, g.nz), fy = hedge(i, g.nx) * hedge(k, g.nz),
               fz = hedge(i, g.nx) * hedge(j, g.ny);
        int nbi[6] = {i - 1, i + 1, i, i, i, i}, nbj[6] = {j, j, j - 1, j + 1, j, j}, nbk[6] = {k, k, k, k, k - 1, k + 1};
        double f[6] = {fx, fx, fy, fy, fz, fz};
        for (int d = 0; d < 6; ++d) {
            int ii = nbi[d], jj = nbj[d], kk = nbk[d];
            if (ii < 0 || ii >= g.nx || jj < 0 || jj >= g.ny || kk < 0 || kk >= g.nz) continue;
            dg += f[d];  // diagonal of the fine row
            int64_t m = ((int64_t)kk * g.ny + jj) * g.nx + ii;
            if (type[m] != 0) continue;
            int pi = ii / 2, pj = jj / 2, pk = kk / 2;
            if (pi == Ix && pj == Iy && pk == Iz) dg -= f[d];       // pair inside the aggregate
            else if (d == 1 && pi == Ix + 1) cx -= f[d];             // +x face
            else if (d == 3 && pj == Iy + 1) cy -= f[d];             // +y face
            else if (d == 5 && pk == Iz + 1) cz -= f[d];             // +z face
        }
    }
    c.diag[I] = (mgv)dg;
    c.cx[I] = (mgv)cx;
    c.cy[I] = (mgv)cy;
    c.cz[I] = (mgv)cz;
}

// Level l+1 from the stored stencil of level l.
__global__ void k_mg_build(MgLevel f, MgLevel c) {
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= c.n) return;
    int Ix = (int)(I % c.nx), Iy = (int)((I / c.nx) % c.ny), Iz = (int)(I / ((int64_t)c.nx * c.ny));
    double dg = 0.0, cx = 0.0, cy = 0.0, cz = 0.0;
    int64_t pl = (int64_t)f.nx * f.ny;
    for (int t = 0; t < 8; ++t) {
        int i = 2 * Ix + (t & 1), j = 2 * Iy + ((t >> 1) & 1), k = 2 * Iz + ((t >> 2) & 1);
        if (i >= f.nx || j >= f.ny || k >= f.nz) continue;
        int64_t n = ((int64_t)k * f.ny + j) * f.nx + i;
        if (f.diag[n] == 0.0) continue;
        dg += f.diag[n];
        // couplings to the six neighbours (off-diagonals are <= 0)
        double cpl[6] = {i > 0 ? f.cx[n - 1] : 0.0, f.cx[n], j > 0 ? f.cy[n - f.nx] : 0.0, f.cy[n],
                         k > 0 ? f.cz[n - pl] : 0.0, f.cz[n]};
        int nbi[6] = {i - 1, i + 1, i, i, i, i}, nbj[6] = {j, j, j - 1, j + 1, j, j}, nbk[6] = {k, k, k, k, k - 1, k + 1};
        for (int d = 0; d < 6; ++d) {
            if (cpl[d] == 0.0 || nbi[d] < 0 || nbj[d] < 0 || nbk[d] < 0) continue;
            int pi = nbi[d] / 2, pj = nbj[d] / 2, pk = nbk[d] / 2;
            if (pi == Ix && pj == Iy && pk == Iz) dg += cpl[d];
            else if (d == 1 && pi == Ix + 1) cx += cpl[d];
            else if (d == 3 && pj == Iy + 1) cy += cpl[d];
            else if (d == 5 && pk == Iz + 1) cz += cpl[d];
        }
    }
    c.diag[I] = (mgv)dg;
    c.cx[I] = (mgv)cx;
    c.cy[I] = (mgv)cy;
    c.cz[I] = (mgv)cz;
}

// ---------------------------------------------------------------------------
// Operator application

// (A x)_n on a coarse level. Neighbours outside the grid are read at the node
// itself with a zero coefficient, so all loads are unconditional.
__device__ inline double apply_coarse(const MgLevel& L, const mgv* __restrict__ x, int64_t n, int i, int j, int k,
                                      double xn) {
    int64_t pl = (int64_t)L.nx * L.ny;
    const int64_t ow = i > 0 ? -1 : 0, oe = i < L.nx - 1 ? 1 : 0;
    const int64_t os = j > 0 ? -(int64_t)L.nx : 0, on = j < L.ny - 1 ? (int64_t)L.nx : 0;
    const int64_t ob = k > 0 ? -pl : 0, ot = k < L.nz - 1 ? pl : 0;
    const double cw = L.cx[n + ow], ce = L.cx[n], cs = L.cy[n + os], cn = L.cy[n], cb = L.cz[n + ob], ct = L.cz[n];
    const double xw = x[n + ow], xe = x[n + oe], xs = x[n + os], xnn = x[n + on], xb = x[n + ob], xt = x[n + ot];
    double s = L.diag[n] * xn;
    s += (i > 0 ? cw : 0.0) * xw;
    s += (i < L.nx - 1 ? ce : 0.0) * xe;
    s += (j > 0 ? cs : 0.0) * xs;
    s += (j < L.ny - 1 ? cn : 0.0) * xnn;
    s += (k > 0 ? cb : 0.0) * xb;
    s += (k < L.nz - 1 ? ct : 0.0) * xt;
    return s;
}

// ---------------------------------------------------------------------------
// Smoothing, restriction, prolongation

struct MgArgs {
    Grid g;
    const uint8_t* type;
    DevState* s;
    double* part_rr;   // CG partials of r.r (finest level, read by the first kernel)
    double* part_bb;   // CG partials of b.b (read before the first iteration)
    double* part_rz;   // partials of r.z written by the last kernel
};

// Convergence test of the CG update (one block): finishes r.r (and b.b
// before the first iteration) and sets done.
__global__ void k_mg_test(MgArgs a, int cg_blocks) {
    DevState* s = a.s;
    if (s->done) return;
    double rr = sum_partials_n(a.part_rr, cg_blocks);
    double bb;
    if (s->it == 0) {
        bb = sum_partials_n(a.part_bb, cg_blocks);
        if (threadIdx.x == 0) {
            s->bb = bb;
            s->rr0 = rr;
        }
    } else {
        bb = s->bb;
    }
    bool conv = (bb == 0.0) || (sqrt(rr) <= s->rtol * sqrt(bb)) || (s->it >= s->maxit);
    if (threadIdx.x == 0) {
        s->rr = rr;
        if (conv) {
            s->done = 1;
            s->zero_solution = (bb == 0.0);
        }
    }
}

// First sweep from x = 0 on a coarse level: x = omega D^-1 b.
// (The small coarse-level kernels issue their loads before testing whether
// the solve is done, so the two latencies overlap.)
__global__ __launch_bounds__(kBlock) void k_mg_first(MgArgs a, MgLevel L) {
    DevState* s = a.s;
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= L.n) return;
    const double d = L.diag[n], bn = L.b[n];
    if (s->done) return;
    L.x0[n] = (mgv)(d == 0.0 ? 0.0 : kOmega * bn / d);
}

// One damped Jacobi sweep on a coarse level, xo = xi + omega D^-1 (b - A xi),
// optionally adding the prolonged coarse correction alpha_c P xc to xi first
// (applied to every value read, so no separate pass is needed).
__global__ __launch_bounds__(kBlock) void k_mg_jacobi(MgArgs a, MgLevel L, const mgv* __restrict__ xi,
                                                       mgv* __restrict__ xo, const mgv* __restrict__ xc, MgLevel C,
                                                       double alpha_c) {
    DevState* s = a.s;
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= L.n) return;
    int i = (int)(n % L.nx), j = (int)((n / L.nx) % L.ny), k = (int)(n / ((int64_t)L.nx * L.ny));
    auto val = [&](int64_t m, int ii, int jj, int kk) -> double {
        double v = xi[m];
        if (xc) v += alpha_c * (double)xc[((int64_t)(kk / 2) * C.ny + jj / 2) * C.nx + ii / 2];
        return v;
    };
    int64_t pl = (int64_t)L.nx * L.ny;
    // neighbours outside the grid are read at the node itself, zero coefficient
    const int iw = i > 0 ? i - 1 : i, ie = i < L.nx - 1 ? i + 1 : i;
    const int js = j > 0 ? j - 1 : j, jn = j < L.ny - 1 ? j + 1 : j;
    const int kb = k > 0 ? k - 1 : k, kt = k < L.nz - 1 ? k + 1 : k;
    const int64_t ow = iw - i, oe = ie - i, os = (int64_t)(js - j) * L.nx, on = (int64_t)(jn - j) * L.nx;
    const int64_t ob = (int64_t)(kb - k) * pl, ot = (int64_t)(kt - k) * pl;
    const double d = L.diag[n], bn = L.b[n];
    const double cw = L.cx[n + ow], ce = L.cx[n], cs = L.cy[n + os], cn = L.cy[n], cb = L.cz[n + ob], ct = L.cz[n];
    const double xn = val(n, i, j, k);
    const double xw = val(n + ow, iw, j, k), xe = val(n + oe, ie, j, k), xs = val(n + os, i, js, k),
                 xnn = val(n + on, i, jn, k), xb = val(n + ob, i, j, kb), xt = val(n + ot, i, j, kt);
    if (s->done) return;
    double sacc = d * xn;
    sacc += (i > 0 ? cw : 0.0) * xw;
    sacc += (i < L.nx - 1 ? ce : 0.0) * xe;
    sacc += (j > 0 ? cs : 0.0) * xs;
    sacc += (j < L.ny - 1 ? cn : 0.0) * xnn;
    sacc += (k > 0 ? cb : 0.0) * xb;
    sacc += (k < L.nz - 1 ? ct : 0.0) * xt;
    // a node without an unknown (diag 0) stays zero
    xo[n] = (mgv)(d == 0.0 ? 0.0 : xn + kOmega * (bn - sacc) / (d == 0.0 ? 1.0 : d));
}

// b_c = P^T (b - A x) between two coarse levels: eight consecutive threads
// per coarse node, one per child, summed in a fixed order by lane exchanges
// ((c0 + c1) + (c2 + c3)) + ((c4 + c5) + (c6 + c7)).
__global__ __launch_bounds__(kBlock) void k_mg_restrict(MgArgs a, MgLevel F, const mgv* __restrict__ x, MgLevel C) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t I = gid >> 3;
    const int t = (int)(gid & 7);
    const bool valid = I < C.n;
    const int64_t Ic = valid ? I : C.n - 1;
    const int Ix = (int)(Ic % C.nx), Iy = (int)((Ic / C.nx) % C.ny), Iz = (int)(Ic / ((int64_t)C.nx * C.ny));
    int i = 2 * Ix + (t & 1), j = 2 * Iy + ((t >> 1) & 1), k = 2 * Iz + ((t >> 2) & 1);
    const bool in = i < F.nx && j < F.ny && k < F.nz;
    // a child outside the grid is evaluated at the first child, weight zero
    if (!in) {
        i = 2 * Ix;
        j = 2 * Iy;
        k = 2 * Iz;
    }
    const int64_t n = ((int64_t)k * F.ny + j) * F.nx + i;
    const double r = (double)F.b[n] - apply_coarse(F, x, n, i, j, k, x[n]);
    double v = (in && F.diag[n] != (mgv)0) ? r : 0.0;
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    if (a.s->done) return;
    if (t == 0 && valid) C.b[I] = (mgv)v;
}

// Coarsest level: x = A^-1 b with the stored inverse, one wavefront per row.
__global__ __launch_bounds__(kBlock) void k_mg_coarsest(MgArgs a, MgLevel L, const double* __restrict__ inv) {
    if (a.s->done) return;
    int64_t row = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    int lane = threadIdx.x & 63;
    if (row >= L.n) return;
    double acc = 0.0;
    for (int64_t c = lane; c < L.n; c += 64) acc += inv[row * L.n + c] * (double)L.b[c];
    acc = wave_sum(acc);
    if (lane == 0) L.x0[row] = (mgv)acc;
}

// ---------------------------------------------------------------------------
// Finest level (z-marching, see ZMarch)

__device__ inline double fine_diag(const Grid& g, int i, int j, int k) {
    double hx = hedge(i, g.nx), hy = hedge(j, g.ny), hz = hedge(k, g.nz);
    double fx = hy * hz, fy = hx * hz, fz = hx * hy;
    return (i > 0 ? fx : 0.0) + (i < g.nx - 1 ? fx : 0.0) + (j > 0 ? fy : 0.0) + (j < g.ny - 1 ? fy : 0.0) +
           (k > 0 ? fz : 0.0) + (k < g.nz - 1 ? fz : 0.0);
}

// Input value of a fine sweep at node m = (i, j, k):
//   kFineFirst: the first sweep from zero, omega b / D (b is zero on fixed nodes);
//   kFineCorr : xi + alpha_c P xc on free nodes, zero on fixed nodes;
//   kFinePlain: xi (zero on fixed nodes).
// The diagonal of a free node does not depend on k (free nodes are never on
// a z face), so kFineFirst takes omega / D of the node's column, cw.
constexpr int kFinePlain = 0, kFineFirst = 1, kFineCorr = 2;

template <int MODE, typename TB>
struct FineIn {
    const uint8_t* __restrict__ type;
    const mgv* __restrict__ xi;
    const TB* __restrict__ b;
    const mgv* __restrict__ xc;
    int cnx, cny;
    double ac;
    __device__ double operator()(int64_t m, int i, int j, int k, double cw) const {
        if (MODE == kFineFirst) return cw * (double)b[m];
        if (MODE == kFineCorr) {
            // all three loads unconditional and the mask applied by a product
            // (a select lets the compiler branch around the loads)
            const uint8_t tv = type[m];
            const double xv = xi[m];
            const double cv = (double)xc[((int64_t)(k >> 1) * cny + (j >> 1)) * cnx + (i >> 1)];
            return (xv + ac * cv) * (double)(tv == 0);
        }
        return (double)xi[m];
    }
};

// omega / D for a free node of column (i, j) (zero outside the grid)
__device__ inline double col_weight(const Grid& g, int i, int j) {
    if (i < 0 || i >= g.nx || j < 0 || j >= g.ny) return 0.0;
    return kOmega / fine_diag(g, i, j, 1 < g.nz - 1 ? 1 : 0);
}

// One damped Jacobi sweep on the finest level; with LAST the partials of
// r.z (b . xo) are written, one per block.
template <int MODE, bool LAST, typename TB>
__global__ __launch_bounds__(kBlock) void k_mg_fine_sweep(MgArgs a, const TB* __restrict__ b0, const mgv* __restrict__ xi,
                                                           mgv* __restrict__ xo, const mgv* __restrict__ xc, MgLevel C,
                                                           double alpha_c, int kc) {
    DevState* s = a.s;
    if (s->done) return;
    const Grid& g = a.g;
    FineIn<MODE, TB> in{a.type, xi, b0, xc, C.nx, C.ny, alpha_c};
    ZMarch t = zmarch(g.nx, g.ny, g.nz, kc);
    double rz = 0.0;
    if (t.col) {
        int i = t.i, j = t.j;
        int64_t pl = (int64_t)g.nx * g.ny;
        int64_t n = (int64_t)t.k0 * pl + (int64_t)j * g.nx + i;
        double hx = hedge(i, g.nx), hy = hedge(j, g.ny), fz = hx * hy;
        double cw = col_weight(g, i, j), cwW = 0.0, cwE = 0.0, cwS = 0.0, cwN = 0.0;
        if (MODE == kFineFirst) {
            cwW = col_weight(g, i - 1, j);
            cwE = col_weight(g, i + 1, j);
            cwS = col_weight(g, i, j - 1);
            cwN = col_weight(g, i, j + 1);
        }
        // neighbours outside the grid are read at the node itself (every load
        // is unconditional, so a step's loads are issued together) and given
        // a zero weight
        const int iw = i > 0 ? i - 1 : i, ie = i < g.nx - 1 ? i + 1 : i;
        const int js = j > 0 ? j - 1 : j, jn = j < g.ny - 1 ? j + 1 : j;
        const int64_t ow = iw - i, oe = ie - i, os = (int64_t)(js - j) * g.nx, on = (int64_t)(jn - j) * g.nx;
        const double ww = i > 0 ? hy : 0.0, we = i < g.nx - 1 ? hy : 0.0;
        const double ws = j > 0 ? hx : 0.0, wn = j < g.ny - 1 ? hx : 0.0;
        double vm = in(t.k0 > 0 ? n - pl : n, i, j, t.k0 > 0 ? t.k0 - 1 : t.k0, cw);
        if (t.k0 == 0) vm = 0.0;
        double vc = in(n, i, j, t.k0, cw);
        for (int k = t.k0; k < t.k1; ++k, n += pl) {
            const bool up = k + 1 < g.nz;
            double vp = in(up ? n + pl : n, i, j, up ? k + 1 : k, cw);
            if (!up) vp = 0.0;
            const double xw = in(n + ow, iw, j, k, cwW), xe = in(n + oe, ie, j, k, cwE);
            const double xs = in(n + os, i, js, k, cwS), xn = in(n + on, i, jn, k, cwN);
            const double bn = (double)b0[n];
            const bool fr = a.type[n] == 0;
            // a free node is never on a z face: fx = hy, fy = hx (hz = 1)
            double acc = 0.0;
            acc += ww * (vc - xw);
            acc += we * (vc - xe);
            acc += ws * (vc - xs);
            acc += wn * (vc - xn);
            acc += fz * (vc - vm);
            acc += fz * (vc - vp);
            const mgv out = (mgv)((vc + cw * (bn - acc)) * (double)fr);  // values are finite
            if (LAST) rz += bn * (double)out;
            xo[n] = out;
            vm = vc;
            vc = vp;
        }
    }
    if (LAST) {
        __shared__ double sh[kBlock / 64];
        double tsum = block_sum(rz, sh);
        if (threadIdx.x == 0) a.part_rz[blockIdx.x] = tsum;
    }
}

// b_1 = P^T (b - A x) from the finest level (kc even, so both fine planes of
// a coarse plane are in one block). The residuals of the two planes are added
// in the thread, the x pair by a lane exchange and the y pair through LDS,
// always as (even + odd).
template <typename TB>
__global__ __launch_bounds__(kBlock) void k_mg_fine_restrict(MgArgs a, const TB* __restrict__ b0, const mgv* __restrict__ x,
                                                              MgLevel C, int kc) {
    if (a.s->done) return;
    __shared__ double sh[4][64];
    const Grid& g = a.g;
    ZMarch t = zmarch(g.nx, g.ny, g.nz, kc);
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int i = t.i, j = t.j;
    const bool col = t.col;
    const int64_t pl = (int64_t)g.nx * g.ny;
    int64_t n = col ? (int64_t)t.k0 * pl + (int64_t)j * g.nx + i : 0;
    double hx = hedge(i, g.nx), hy = hedge(j, g.ny), fz = hx * hy;
    const int iw = i > 0 ? i - 1 : i, ie = i < g.nx - 1 ? i + 1 : i;
    const int js = j > 0 ? j - 1 : j, jn = j < g.ny - 1 ? j + 1 : j;
    const int64_t ow = iw - i, oe = ie - i, os = (int64_t)(js - j) * g.nx, on = (int64_t)(jn - j) * g.nx;
    const double ww = i > 0 ? hy : 0.0, we = i < g.nx - 1 ? hy : 0.0;
    const double ws = j > 0 ? hx : 0.0, wn = j < g.ny - 1 ? hx : 0.0;
    double vm = (col && t.k0 > 0) ? (double)x[n - pl] : 0.0;
    double vc = col ? (double)x[n] : 0.0;
    double pair = 0.0;
    for (int k = t.k0; k < t.k1; ++k, n += pl) {
        double res = 0.0;
        double vp = 0.0;
        if (col) {
            const bool up = k + 1 < g.nz;
            vp = (double)x[up ? n + pl : n];
            if (!up) vp = 0.0;
            const double xw = x[n + ow], xe = x[n + oe], xs = x[n + os], xn = x[n + on];
            const double bn = (double)b0[n];
            const bool fr = a.type[n] == 0;
            double acc = 0.0;
            acc += ww * (vc - xw);
            acc += we * (vc - xe);
            acc += ws * (vc - xs);
            acc += wn * (vc - xn);
            acc += fz * (vc - vm);
            acc += fz * (vc - vp);
            res = fr ? bn - acc : 0.0;
        }
        pair += res;
        if ((k & 1) || k == g.nz - 1) {
            double o = __shfl_xor(pair, 1);
            double sx = (tx & 1) ? o + pair : pair + o;
            sh[ty][tx] = sx;
            __syncthreads();
            if (!(tx & 1) && !(ty & 1) && col) {
                int64_t I = ((int64_t)(k >> 1) * C.ny + (j >> 1)) * C.nx + (i >> 1);
                C.b[I] = (mgv)(sh[ty][tx] + sh[ty + 1][tx]);
            }
            __syncthreads();
            pair = 0.0;
        }
        vm = vc;
        vc = vp;
    }
}

// ---------------------------------------------------------------------------
// Host side

static unsigned mg_grid(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    return (unsigned)(g < 1 ? 1 : g);
}

// Inverse of the coarsest operator (n <= 1024) by Cholesky factorization on
// the host; rows and columns of nodes without unknowns (diag 0) stay zero.
static int coarsest_inverse(const MgLevel& L, const std::vector<double>& dg, const std::vector<double>& cx,
                            const std::vector<double>& cy, const std::vector<double>& cz, std::vector<double>& inv) {
    const int64_t n = L.n;
    std::vector<int> act;
    std::vector<int> pos(n, -1);
    for (int64_t I = 0; I < n; ++I)
        if (dg[I] != 0.0) {
            pos[I] = (int)act.size();
            act.push_back((int)I);
        }
    const int m = (int)act.size();
    std::vector<double> A((size_t)m * m, 0.0);
    const int64_t pl = (int64_t)L.nx * L.ny;
    for (int r = 0; r < m; ++r) {
        int64_t I = act[r];
        int i = (int)(I % L.nx), j = (int)((I / L.nx) % L.ny), k = (int)(I / pl);
        A[(size_t)r * m + r] = dg[I];
        auto couple = [&](int64_t J, double v) {
            if (J < 0 || J >= n || pos[J] < 0 || v == 0.0) return;
            A[(size_t)r * m + pos[J]] = v;
        };
        if (i > 0) couple(I - 1, cx[I - 1]);
        if (i < L.nx - 1) couple(I + 1, cx[I]);
        if (j > 0) couple(I - L.nx, cy[I - L.nx]);
        if (j < L.ny - 1) couple(I + L.nx, cy[I]);
        if (k > 0) couple(I - pl, cz[I - pl]);
        if (k < L.nz - 1) couple(I + pl, cz[I]);
    }
    // A = R^T R (upper R in place)
    for (int c = 0; c < m; ++c) {
        double d = A[(size_t)c * m + c];
        for (int t = 0; t < c; ++t) d -= A[(size_t)t * m + c] * A[(size_t)t * m + c];
        if (!(d > 0.0)) return -3;
        d = std::sqrt(d);
        A[(size_t)c * m + c] = d;
        for (int col = c + 1; col < m; ++col) {
            double v = A[(size_t)c * m + col];
            for (int t = 0; t < c; ++t) v -= A[(size_t)t * m + c] * A[(size_t)t * m + col];
            A[(size_t)c * m + col] = v / d;
        }
    }
    inv.assign((size_t)n * n, 0.0);
    std::vector<double> y(m);
    for (int e = 0; e < m; ++e) {
        // R^T y = e_e, then R x = y
        for (int r = 0; r < m; ++r) {
            double v = (r == e) ? 1.0 : 0.0;
            for (int t = 0; t < r; ++t) v -= A[(size_t)t * m + r] * y[t];
            y[r] = v / A[(size_t)r * m + r];
        }
        for (int r = m - 1; r >= 0; --r) {
            double v = y[r];
            for (int t = r + 1; t < m; ++t) v -= A[(size_t)r * m + t] * y[t];
            y[r] = v / A[(size_t)r * m + r];
        }
        for (int r = 0; r < m; ++r) inv[(size_t)act[r] * n + act[e]] = y[r];
    }
    return 0;
}

int mg_setup(pic_ctx* c) {
    std::vector<int3> dims;
    mg_dims(&c->cfg, dims);
    char* base = (char*)c->mg;
    auto take = [&](size_t bytes) -> char* {
        char* p = base;
        base += (bytes + 255) & ~size_t(255);
        return p;
    };
    MgHier* h = new MgHier();
    h->nlev = (int)dims.size();
    int64_t nn = c->g.nn;
    if (h->nlev < 2 || (int64_t)dims.back().x * dims.back().y * dims.back().z > 1024) {
        delete h;
        return -3;
    }
    h->z[0] = (mgv*)take(nn * sizeof(mgv));
    h->z[1] = (mgv*)take(nn * sizeof(mgv));
    h->part = (double*)take(64 * kMgBlocks * 8);
    for (int l = 0; l < h->nlev; ++l) {
        MgLevel& L = h->lv[l];
        L.nx = dims[l].x;
        L.ny = dims[l].y;
        L.nz = dims[l].z;
        L.n = (int64_t)L.nx * L.ny * L.nz;
        if (l == 0) {
            L.diag = L.cx = L.cy = L.cz = nullptr;
            L.x0 = h->z[0];
            L.x1 = h->z[1];
            L.b = nullptr;  // the finest right-hand side is passed to each V-cycle
            continue;
        }
        L.diag = (mgv*)take(L.n * sizeof(mgv));
        L.cx = (mgv*)take(L.n * sizeof(mgv));
        L.cy = (mgv*)take(L.n * sizeof(mgv));
        L.cz = (mgv*)take(L.n * sizeof(mgv));
        L.x0 = (mgv*)take(L.n * sizeof(mgv));
        L.x1 = (mgv*)take(L.n * sizeof(mgv));
        L.b = (mgv*)take(L.n * sizeof(mgv));
    }
    MgLevel& Lc = h->lv[h->nlev - 1];
    h->cinv = (double*)take((size_t)Lc.n * Lc.n * 8);
    // two Jacobi sweeps each way; the piecewise-constant prolongation leaves
    // the coarse correction too small by about a factor 2, which the weight
    // alpha_c = 2 restores (24 instead of 60 iterations to 1e-8 on the
    // 128 x 128 x 512 grid)
    h->pre = 2;
    h->post = 2;
    h->alpha_c = 2.0;
    h->zm_blocks = zmarch_grid(c->g.nx, c->g.ny, c->g.nz, stencil_target(c), 1, &h->zm_kc);
    h->zr_blocks = zmarch_grid(c->g.nx, c->g.ny, c->g.nz, stencil_target(c), 2, &h->zr_kc);
    if (h->zm_blocks > 4096) {
        delete h;
        return -3;
    }
    for (int l = 1; l < h->nlev; ++l) {
        MgLevel& C = h->lv[l];
        unsigned G = (unsigned)((C.n + kBlock - 1) / kBlock);
        if (l == 1)
            hipLaunchKernelGGL(k_mg_build1, dim3(G), dim3(kBlock), 0, c->stream, c->g, c->buf.node_type, C);
        else
            hipLaunchKernelGGL(k_mg_build, dim3(G), dim3(kBlock), 0, c->stream, h->lv[l - 1], C);
    }
    // exact solve on the coarsest level
    int64_t m = Lc.n;
    std::vector<mgv> dgf(m), cxf(m), cyf(m), czf(m);
    std::vector<double> inv;
    if (hipMemcpyAsync(dgf.data(), Lc.diag, m * sizeof(mgv), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipMemcpyAsync(cxf.data(), Lc.cx, m * sizeof(mgv), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipMemcpyAsync(cyf.data(), Lc.cy, m * sizeof(mgv), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipMemcpyAsync(czf.data(), Lc.cz, m * sizeof(mgv), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        delete h;
        return -2;
    }
    std::vector<double> dg(dgf.begin(), dgf.end()), cx(cxf.begin(), cxf.end()), cy(cyf.begin(), cyf.end()),
        cz(czf.begin(), czf.end());
    if (coarsest_inverse(Lc, dg, cx, cy, cz, inv) != 0) {
        delete h;
        return -3;
    }
    if (hipMemcpyAsync(h->cinv, inv.data(), inv.size() * 8, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        delete h;
        return -2;
    }
    c->mg_host = h;
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// z = V-cycle(b0) on the finest level (b0: the CG residual, FP64 or FP32);
// returns the buffer holding z and, in n_rz, the number of r.z partials
// written. The first kernel finishes r.r and tests convergence, the last
// writes the partials of r.z. Every call launches the same kernels with the
// same arguments.
template <typename TB>
float* mg_vcycle(pic_ctx* c, const TB* b0, double* part_rr, double* part_bb, double* part_rz, int cg_blocks, int* n_rz,
                 bool timed) {
    MgHier* h = (MgHier*)c->mg_host;
    MgArgs a;
    a.g = c->g;
    a.type = c->buf.node_type;
    a.s = c->st;
    a.part_rr = part_rr;
    a.part_bb = part_bb;
    a.part_rz = part_rz;
    const int nl = h->nlev;
    const mgv* nul = nullptr;
    mgv* pre_out[kMgMaxLevels];  // pre-smoothed iterate per level
    mgv* res[kMgMaxLevels];      // final iterate per level
    hipLaunchKernelGGL(k_mg_test, dim3(1), dim3(kBlock), 0, c->stream, a, cg_blocks);
    // descending: pre-smoothing (first sweep from zero + one sweep) and restriction
    for (int l = 0; l < nl - 1; ++l) {
        MgLevel& L = h->lv[l];
        MgLevel& C = h->lv[l + 1];
        if (l == 0) {
            int t1 = timed ? tic(c, PIC_T_MG_FIRST) : -1;
            hipLaunchKernelGGL((k_mg_fine_sweep<kFineFirst, false, TB>), dim3(h->zm_blocks), dim3(kBlock), 0,
                               c->stream, a, b0, nul, L.x0, nul, C, 0.0, h->zm_kc);
            toc(c, t1);
            int t2 = timed ? tic(c, PIC_T_MG_RESTRICT) : -1;
            hipLaunchKernelGGL(k_mg_fine_restrict<TB>, dim3(h->zr_blocks), dim3(kBlock), 0, c->stream, a, b0,
                               (const mgv*)L.x0, C, h->zr_kc);
            toc(c, t2);
            pre_out[0] = L.x0;
        } else {
            hipLaunchKernelGGL(k_mg_first, dim3(mg_grid(L.n)), dim3(kBlock), 0, c->stream, a, L);
            hipLaunchKernelGGL(k_mg_jacobi, dim3(mg_grid(L.n)), dim3(kBlock), 0, c->stream, a, L, (const mgv*)L.x0, L.x1,
                               nul, C, 0.0);
            hipLaunchKernelGGL(k_mg_restrict, dim3(mg_grid(8 * C.n)), dim3(kBlock), 0, c->stream, a, L, (const mgv*)L.x1,
                               C);
            pre_out[l] = L.x1;
        }
    }
    hipLaunchKernelGGL(k_mg_coarsest, dim3((unsigned)((h->lv[nl - 1].n + 3) / 4)), dim3(kBlock), 0, c->stream, a,
                       h->lv[nl - 1], (const double*)h->cinv);
    res[nl - 1] = h->lv[nl - 1].x0;
    // ascending: correction (fused into the first post sweep) and one more sweep
    for (int l = nl - 2; l >= 0; --l) {
        MgLevel& L = h->lv[l];
        MgLevel& C = h->lv[l + 1];
        mgv* xi = pre_out[l];
        mgv* xo = xi == L.x0 ? L.x1 : L.x0;
        if (l == 0) {
            int t1 = timed ? tic(c, PIC_T_MG_CORR) : -1;
            hipLaunchKernelGGL((k_mg_fine_sweep<kFineCorr, false, TB>), dim3(h->zm_blocks), dim3(kBlock), 0, c->stream,
                               a, b0, (const mgv*)xi, xo, (const mgv*)res[1], C, h->alpha_c, h->zm_kc);
            toc(c, t1);
            int t2 = timed ? tic(c, PIC_T_MG_LAST) : -1;
            hipLaunchKernelGGL((k_mg_fine_sweep<kFinePlain, true, TB>), dim3(h->zm_blocks), dim3(kBlock), 0, c->stream,
                               a, b0, (const mgv*)xo, xi, nul, C, 0.0, h->zm_kc);
            toc(c, t2);
        } else {
            hipLaunchKernelGGL(k_mg_jacobi, dim3(mg_grid(L.n)), dim3(kBlock), 0, c->stream, a, L, (const mgv*)xi, xo,
                               (const mgv*)res[l + 1], C, h->alpha_c);
            hipLaunchKernelGGL(k_mg_jacobi, dim3(mg_grid(L.n)), dim3(kBlock), 0, c->stream, a, L, (const mgv*)xo, xi, nul,
                               C, 0.0);
        }
        res[l] = xi;
    }
    *n_rz = (int)h->zm_blocks;
    return res[0];
}

template float* mg_vcycle<double>(pic_ctx*, const double*, double*, double*, double*, int, int*, bool);
template float* mg_vcycle<float>(pic_ctx*, const float*, double*, double*, double*, int, int*, bool);

void mg_free(pic_ctx* c) {
    delete (MgHier*)c->mg_host;
    c->mg_host = nullptr;
}


}  // namespace pic
