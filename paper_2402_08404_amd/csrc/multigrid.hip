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
// a symmetric positive definite preconditioner for CG.
#include <vector>

#include "pic_internal.hpp"

namespace pic {

constexpr int kMgMaxLevels = 12;
constexpr int kMgBlocks = 1024;
constexpr double kOmega = 6.0 / 7.0;  // damped Jacobi weight for 7-point stencils
constexpr int kCoarseSweeps = 64;

struct MgLevel {
    int nx, ny, nz;
    int64_t n;
    double *diag, *cx, *cy, *cz;  // levels >= 1
    double *x0, *x1, *b;          // x ping-pong and right-hand side
};

struct MgHier {
    int nlev;
    MgLevel lv[kMgMaxLevels];
    double* z[2];  // finest-level preconditioned residual (ping-pong)
    double* part;  // partial sums
    int pre, post;
    double alpha_c;
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
    b += 2 * nn * 8 + 64 * kMgBlocks * 8;
    for (size_t l = 1; l < dims.size(); ++l) {
        int64_t n = (int64_t)dims[l].x * dims[l].y * dims[l].z;
        b += 7 * (size_t)n * 8 + 7 * 256;
    }
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
    int64_t pl = (int64_t)g.nx * g.ny;
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
    c.diag[I] = dg;
    c.cx[I] = cx;
    c.cy[I] = cy;
    c.cz[I] = cz;
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
    c.diag[I] = dg;
    c.cx[I] = cx;
    c.cy[I] = cy;
    c.cz[I] = cz;
}

// ---------------------------------------------------------------------------
// Operator application

// Finest level, matrix free: returns (A x)_n and the diagonal. x must be zero
// on nodes held at a fixed potential (true for every multigrid vector).
__device__ inline double apply_fine(const Grid& g, const uint8_t* __restrict__ type, const double* __restrict__ x,
                                    int64_t n, int i, int j, int k, double xn, double* dg) {
    int64_t pl = (int64_t)g.nx * g.ny;
    double fx = hedge(j, g.ny) * hedge(k, g.nz), fy = hedge(i, g.nx) * hedge(k, g.nz), fz = hedge(i, g.nx) * hedge(j, g.ny);
    int64_t nb[6] = {n - 1, n + 1, n - g.nx, n + g.nx, n - pl, n + pl};
    bool has[6] = {i > 0, i < g.nx - 1, j > 0, j < g.ny - 1, k > 0, k < g.nz - 1};
    double f[6] = {fx, fx, fy, fy, fz, fz};
    double acc = 0.0, d = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        if (!has[q]) continue;
        d += f[q];
        acc += f[q] * (xn - x[nb[q]]);
    }
    *dg = d;
    return acc;
}

__device__ inline double apply_coarse(const MgLevel& L, const double* __restrict__ x, int64_t n, int i, int j, int k,
                                      double xn) {
    int64_t pl = (int64_t)L.nx * L.ny;
    double s = L.diag[n] * xn;
    if (i > 0) s += L.cx[n - 1] * x[n - 1];
    if (i < L.nx - 1) s += L.cx[n] * x[n + 1];
    if (j > 0) s += L.cy[n - L.nx] * x[n - L.nx];
    if (j < L.ny - 1) s += L.cy[n] * x[n + L.nx];
    if (k > 0) s += L.cz[n - pl] * x[n - pl];
    if (k < L.nz - 1) s += L.cz[n] * x[n + pl];
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

__device__ inline double sum_parts(const double* part, int nparts) {
    __shared__ double sh[kBlock / 64];
    __shared__ double res;
    double v = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) v += part[i];
    double t = block_sum(v, sh);
    if (threadIdx.x == 0) res = t;
    __syncthreads();
    return res;
}

// Convergence test of the CG update (one block): finishes r.r (and b.b
// before the first iteration) and sets done.
__global__ void k_mg_test(MgArgs a, int cg_blocks) {
    DevState* s = a.s;
    if (s->done) return;
    double rr = sum_parts(a.part_rr, cg_blocks);
    double bb;
    if (s->it == 0) {
        bb = sum_parts(a.part_bb, cg_blocks);
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

// First sweep from x = 0: x = omega D^-1 b.
__global__ __launch_bounds__(kBlock) void k_mg_first(MgArgs a, MgLevel L, int level) {
    DevState* s = a.s;
    if (s->done) return;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    NodeWalk wk((int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int)stride, L.nx, L.ny);
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < L.n; n += stride, wk.advance()) {
        double d;
        if (level == 0) {
            if (a.type[n] != 0) {
                L.x0[n] = 0.0;
                continue;
            }
            const Grid& g = a.g;
            int i = wk.i, j = wk.j, k = wk.k;
            d = (i > 0 ? hedge(j, g.ny) * hedge(k, g.nz) : 0.0) + (i < g.nx - 1 ? hedge(j, g.ny) * hedge(k, g.nz) : 0.0) +
                (j > 0 ? hedge(i, g.nx) * hedge(k, g.nz) : 0.0) + (j < g.ny - 1 ? hedge(i, g.nx) * hedge(k, g.nz) : 0.0) +
                (k > 0 ? hedge(i, g.nx) * hedge(j, g.ny) : 0.0) + (k < g.nz - 1 ? hedge(i, g.nx) * hedge(j, g.ny) : 0.0);
        } else {
            d = L.diag[n];
            if (d == 0.0) {
                L.x0[n] = 0.0;
                continue;
            }
        }
        L.x0[n] = kOmega * L.b[n] / d;
    }
}

// One damped Jacobi sweep xo = xi + omega D^-1 (b - A xi), optionally adding
// the prolonged coarse correction alpha_c P xc to xi first (the correction is
// applied on the fly to every value read, so no separate pass is needed).
// With last != 0 (finest level) the partials of r.z are written.
__global__ __launch_bounds__(kBlock) void k_mg_jacobi(MgArgs a, MgLevel L, int level, const double* __restrict__ xi,
                                                       double* __restrict__ xo, const double* __restrict__ xc,
                                                       MgLevel C, double alpha_c, int last) {
    DevState* s = a.s;
    if (s->done) return;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double rz = 0.0;
    NodeWalk wk((int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int)stride, L.nx, L.ny);
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < L.n; n += stride, wk.advance()) {
        int i = wk.i, j = wk.j, k = wk.k;
        double d, Ax, xn;
        auto val = [&](int64_t m, int ii, int jj, int kk) -> double {
            double v = xi[m];
            if (xc) v += alpha_c * xc[((int64_t)(kk / 2) * C.ny + jj / 2) * C.nx + ii / 2];
            return v;
        };
        int64_t pl = (int64_t)L.nx * L.ny;
        if (level == 0) {
            if (a.type[n] != 0) {
                xo[n] = 0.0;
                continue;
            }
            const Grid& g = a.g;
            double fx = hedge(j, g.ny) * hedge(k, g.nz), fy = hedge(i, g.nx) * hedge(k, g.nz),
                   fz = hedge(i, g.nx) * hedge(j, g.ny);
            xn = val(n, i, j, k);
            double acc = 0.0;
            d = 0.0;
            int64_t nb[6] = {n - 1, n + 1, n - L.nx, n + L.nx, n - pl, n + pl};
            int ni[6] = {i - 1, i + 1, i, i, i, i}, nj[6] = {j, j, j - 1, j + 1, j, j}, nk[6] = {k, k, k, k, k - 1, k + 1};
            bool has[6] = {i > 0, i < L.nx - 1, j > 0, j < L.ny - 1, k > 0, k < L.nz - 1};
            double f[6] = {fx, fx, fy, fy, fz, fz};
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                if (!has[q]) continue;
                d += f[q];
                // the coarse correction reaches free nodes only; without it the
                // iterate is already zero on fixed nodes
                double xj = xc ? (a.type[nb[q]] == 0 ? val(nb[q], ni[q], nj[q], nk[q]) : 0.0) : xi[nb[q]];
                acc += f[q] * (xn - xj);
            }
            Ax = acc;
        } else {
            d = L.diag[n];
            if (d == 0.0) {
                xo[n] = 0.0;
                continue;
            }
            xn = val(n, i, j, k);
            double sacc = d * xn;
            if (i > 0) sacc += L.cx[n - 1] * val(n - 1, i - 1, j, k);
            if (i < L.nx - 1) sacc += L.cx[n] * val(n + 1, i + 1, j, k);
            if (j > 0) sacc += L.cy[n - L.nx] * val(n - L.nx, i, j - 1, k);
            if (j < L.ny - 1) sacc += L.cy[n] * val(n + L.nx, i, j + 1, k);
            if (k > 0) sacc += L.cz[n - pl] * val(n - pl, i, j, k - 1);
            if (k < L.nz - 1) sacc += L.cz[n] * val(n + pl, i, j, k + 1);
            Ax = sacc;
        }
        double bn = L.b[n];
        double xnew = xn + kOmega * (bn - Ax) / d;
        xo[n] = xnew;
        if (last) rz += bn * xnew;
    }
    if (last) {
        __shared__ double sh[kBlock / 64];
        double t = block_sum(rz, sh);
        if (threadIdx.x == 0) a.part_rz[blockIdx.x] = t;
    }
}

// b_c = P^T (b - A x): each coarse node sums the residuals of its children.
__global__ __launch_bounds__(kBlock) void k_mg_restrict(MgArgs a, MgLevel F, int level, const double* __restrict__ x,
                                                         MgLevel C) {
    if (a.s->done) return;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    NodeWalk wk((int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int)stride, C.nx, C.ny);
    for (int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; I < C.n; I += stride, wk.advance()) {
        int Ix = wk.i, Iy = wk.j, Iz = wk.k;
        double sum = 0.0;
        for (int t = 0; t < 8; ++t) {
            int i = 2 * Ix + (t & 1), j = 2 * Iy + ((t >> 1) & 1), k = 2 * Iz + ((t >> 2) & 1);
            if (i >= F.nx || j >= F.ny || k >= F.nz) continue;
            int64_t n = ((int64_t)k * F.ny + j) * F.nx + i;
            double Ax;
            if (level == 0) {
                if (a.type[n] != 0) continue;
                double d;
                Ax = apply_fine(a.g, a.type, x, n, i, j, k, x[n], &d);
            } else {
                if (F.diag[n] == 0.0) continue;
                Ax = apply_coarse(F, x, n, i, j, k, x[n]);
            }
            sum += F.b[n] - Ax;
        }
        C.b[I] = sum;
    }
}

// Coarsest level: kCoarseSweeps damped Jacobi sweeps from zero in one block.
__global__ __launch_bounds__(1024) void k_mg_coarsest(MgArgs a, MgLevel L) {
    if (a.s->done) return;
    __shared__ double xs[2][1024];
    int64_t n = threadIdx.x;
    bool act = n < L.n && L.diag[n] != 0.0;
    double bn = n < L.n ? L.b[n] : 0.0;
    double d = act ? L.diag[n] : 1.0;
    xs[0][threadIdx.x] = 0.0;
    __syncthreads();
    for (int it = 0; it < kCoarseSweeps; ++it) {
        const double* xi = xs[it & 1];
        double* xo = xs[(it + 1) & 1];
        if (n < L.n) {
            double v = 0.0;
            if (act) {
                int ci = (int)(n % L.nx), cj = (int)((n / L.nx) % L.ny), ck = (int)(n / ((int64_t)L.nx * L.ny));
                double Ax = apply_coarse(L, xi, n, ci, cj, ck, xi[n]);
                v = xi[n] + kOmega * (bn - Ax) / d;
            }
            xo[n] = v;
        }
        __syncthreads();
    }
    if (n < L.n) L.x0[n] = xs[kCoarseSweeps & 1][n];
}

// ---------------------------------------------------------------------------
// Host side

// One node per thread, except for the kernel that writes partial sums (a
// fixed number of blocks, as many as the CG kernels read).
static unsigned mg_grid(int64_t n, bool partials) {
    if (partials) return kMgBlocks;
    int64_t g = (n + kBlock - 1) / kBlock;
    return (unsigned)(g < 1 ? 1 : g);
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
    h->z[0] = (double*)take(nn * 8);
    h->z[1] = (double*)take(nn * 8);
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
            L.b = c->cg_r;
            continue;
        }
        L.diag = (double*)take(L.n * 8);
        L.cx = (double*)take(L.n * 8);
        L.cy = (double*)take(L.n * 8);
        L.cz = (double*)take(L.n * 8);
        L.x0 = (double*)take(L.n * 8);
        L.x1 = (double*)take(L.n * 8);
        L.b = (double*)take(L.n * 8);
    }
    // two Jacobi sweeps each way; the piecewise-constant prolongation leaves
    // the coarse correction too small by about a factor 2, which the weight
    // alpha_c = 2 restores (24 instead of 60 iterations to 1e-8 on the
    // 128 x 128 x 512 grid)
    h->pre = 2;
    h->post = 2;
    h->alpha_c = 2.0;
    for (int l = 1; l < h->nlev; ++l) {
        MgLevel& C = h->lv[l];
        unsigned G = (unsigned)((C.n + kBlock - 1) / kBlock);
        if (l == 1)
            hipLaunchKernelGGL(k_mg_build1, dim3(G), dim3(kBlock), 0, c->stream, c->g, c->buf.node_type, C);
        else
            hipLaunchKernelGGL(k_mg_build, dim3(G), dim3(kBlock), 0, c->stream, h->lv[l - 1], C);
    }
    if (h->lv[h->nlev - 1].n > 1024) {
        delete h;
        return -3;
    }
    c->mg_host = h;
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// z = V-cycle(r) on the finest level; returns the buffer holding z. The
// first kernel finishes r.r and tests convergence, the last writes the
// partials of r.z.
double* mg_vcycle(pic_ctx* c, double* part_rr, double* part_bb, double* part_rz, int cg_blocks) {
    MgHier* h = (MgHier*)c->mg_host;
    MgArgs a;
    a.g = c->g;
    a.type = c->buf.node_type;
    a.s = c->st;
    a.part_rr = part_rr;
    a.part_bb = part_bb;
    a.part_rz = part_rz;
    int nl = h->nlev;
    // descending: pre-smoothing and restriction
    for (int l = 0; l < nl - 1; ++l) {
        MgLevel& L = h->lv[l];
        if (l == 0) hipLaunchKernelGGL(k_mg_test, dim3(1), dim3(kBlock), 0, c->stream, a, cg_blocks);
        hipLaunchKernelGGL(k_mg_first, dim3(mg_grid(L.n, false)), dim3(kBlock), 0, c->stream, a, L, l);
        double* xi = L.x0;
        double* xo = L.x1;
        for (int s = 1; s < h->pre; ++s) {
            hipLaunchKernelGGL(k_mg_jacobi, dim3(mg_grid(L.n, false)), dim3(kBlock), 0, c->stream, a, L, l, xi, xo,
                               (const double*)nullptr, h->lv[l + 1], 0.0, 0);
            std::swap(xi, xo);
        }
        // the pre-smoothed iterate must sit in x0 for the way up
        if (xi != L.x0) std::swap(L.x0, L.x1);
        hipLaunchKernelGGL(k_mg_restrict, dim3(mg_grid(h->lv[l + 1].n, false)), dim3(kBlock), 0, c->stream, a, L, l, L.x0,
                           h->lv[l + 1]);
    }
    hipLaunchKernelGGL(k_mg_coarsest, dim3(1), dim3(1024), 0, c->stream, a, h->lv[nl - 1]);
    // ascending: correction (fused into the first post sweep) and smoothing
    double* out = nullptr;
    for (int l = nl - 2; l >= 0; --l) {
        MgLevel& L = h->lv[l];
        double* xi = L.x0;
        double* xo = L.x1;
        for (int s = 0; s < h->post; ++s) {
            bool last = (l == 0) && (s == h->post - 1);
            hipLaunchKernelGGL(k_mg_jacobi, dim3(mg_grid(L.n, last)), dim3(kBlock), 0, c->stream, a, L, l, xi, xo,
                               s == 0 ? (const double*)h->lv[l + 1].x0 : (const double*)nullptr, h->lv[l + 1],
                               h->alpha_c, last ? 1 : 0);
            std::swap(xi, xo);
        }
        if (xi != L.x0) std::swap(L.x0, L.x1);
        out = L.x0;
    }
    return out;
}

void mg_free(pic_ctx* c) {
    delete (MgHier*)c->mg_host;
    c->mg_host = nullptr;
}

int mixed_solve(pic_ctx*, double*, double, const int64_t*, int, double, int, pic_solve_info*) { return -3; }

}  // namespace pic
