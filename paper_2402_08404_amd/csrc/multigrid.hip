// multigrid.hip -- CG preconditioned by a multigrid V-cycle for the
// finite-volume Poisson operator of Eq. poi.
//
// Hierarchy: cell-centred coarsening, each coarse node standing for the (up
// to) 2x2x2 nodes below it. The prolongation P is the cell-centred trilinear
// interpolation (along each axis a node takes 3/4 of its own coarse node and
// 1/4 of the next one on its side; at the grid edge all of its own), the
// restriction is P^T and the coarse operator the Galerkin product P^T A P, a
// stencil of at most 5x5x5 points. Nodes held at a fixed potential are not
// unknowns; a coarse node is an unknown when one of its 2x2x2 nodes is, and
// P has no columns for the others (the interpolated correction tends to zero
// towards a fixed region).
//
// Storage of a coarse operator: the rows of P^T A P are formed in FP64 on the
// device at set-up, rounded to FP32 and grouped on the host into classes of
// identical rows; each node keeps a class id and the level a table of the
// distinct rows (away from the tip and the grid faces almost every node has
// the same row, so a sweep reads the coefficients from cache, not HBM).
// The finest level uses the 7-point operator matrix-free from the node types
// and runs as z-marching kernels.
//
// Smoother: damped Jacobi, the same number of sweeps before and after the
// coarse correction (the first from zero), so the V-cycle is a symmetric
// positive definite preconditioner for CG. The coarsest level (at most
// kCoarseMax nodes) is solved exactly with its inverse, formed once at set-up
// on the device (Gauss-Jordan in FP64) and stored in FP32.
#include <cmath>
#include <cstring>
#include <unordered_map>
#include <vector>

#include "pic_internal.hpp"

namespace pic {

constexpr int kMgMaxLevels = 12;
constexpr int64_t kCoarseMax = 2048;  // nodes of the coarsest level at most

// Storage of every multigrid vector and coarse coefficient: FP32 (the V-cycle
// is a preconditioner, so its precision decides only how good the search
// directions are; the Krylov vectors, dot products and the convergence test
// stay FP64). Arithmetic inside the kernels is FP64.
typedef float mgv;
// Finest level: two Jacobi sweeps before and after the coarse correction with
// the weights 1 / theta_1, 1 / theta_2, theta_i the roots of the degree-2
// Chebyshev polynomial on [0.4, 2] (the eigenvalues of D^-1 A of the 7-point
// operator lie in [0, 2]): the pair multiplies the error components with
// eigenvalues in [0.4, 2] by at most 1 / T_2(1.5) = 0.29 per smoothing,
// against 0.51 for two sweeps with the weight 6/7, and every component with
// an eigenvalue in (0, 2] by less than 1. The two sweeps commute, so the
// V-cycle stays symmetric (before: omega_1 then omega_2; after: omega_2 then
// omega_1).
constexpr double kChebMid = 1.2, kChebHalf = 0.8, kSqrtHalf = 0.70710678118654752;
constexpr double kOmega1 = 1.0 / (kChebMid + kChebHalf * kSqrtHalf);  // 0.5664
constexpr double kOmega2 = 1.0 / (kChebMid - kChebHalf * kSqrtHalf);  // 1.5765
constexpr double kOmegaC = 0.7;         // damped Jacobi weight, 125-point coarse operators
constexpr int kTabRow = 128;            // table row: 125 coefficients, omega / D, row sum
constexpr int kTabInvD = 125;
constexpr int kTabSum = 126;
constexpr int kCenter = 62;             // coefficient index of the node itself

struct MgLevel {
    int nx, ny, nz;
    int64_t n;
    uint32_t* id;   // levels >= 1: row class per node (class 0: no unknown, zero row)
    uint8_t* used;  // levels >= 1: 1 where the node is an unknown
    float* tab;     // levels >= 1: class table, kTabRow values per class
    int ncls;
    mgv *x0, *x1, *b;  // iterates and right-hand side (b: levels >= 1)
    int zkc;           // planes per block of the z-marching sweep (0: plane kernel)
    unsigned zblocks;
};

struct MgHier {
    int nlev;
    MgLevel lv[kMgMaxLevels];
    mgv* z[2];     // finest-level iterates (ping-pong)
    float* cinv;   // inverse of the coarsest operator, n x n (zero rows / columns for non-unknowns)
    int pre, post; // sweeps on the coarse levels (the finest level always does two and two)
    int zm_kc;     // planes per block of the fine sweeps
    unsigned zm_blocks;
    int rz_kc;     // coarse planes per block of the z-marching restriction to level 1
    unsigned rz_blocks;  // its grid (0: the plane kernel)
};

static void mg_dims(const pic_config* cfg, std::vector<int3>& dims) {
    int nx = cfg->nx, ny = cfg->ny, nz = cfg->nz;
    dims.push_back(make_int3(nx, ny, nz));
    while ((int)dims.size() < kMgMaxLevels) {
        int3 d = dims.back();
        const int64_t n = (int64_t)d.x * d.y * d.z;
        // stop at the first coarse level of at most kCoarseMax nodes (a
        // finest grid of at most 512 nodes gets no coarse level)
        if ((n <= kCoarseMax && (dims.size() > 1 || n <= 512)) || d.x <= 2 || d.y <= 2 || d.z <= 2) break;
        dims.push_back(make_int3((d.x + 1) / 2, (d.y + 1) / 2, (d.z + 1) / 2));
    }
}

size_t mg_bytes(const pic_config* cfg) {
    std::vector<int3> dims;
    mg_dims(cfg, dims);
    size_t b = 4096 + sizeof(MgHier);
    int64_t nn = (int64_t)cfg->nx * cfg->ny * cfg->nz;
    b += 2 * nn * sizeof(mgv) + 2 * 256;
    for (size_t l = 1; l < dims.size(); ++l) {
        int64_t n = (int64_t)dims[l].x * dims[l].y * dims[l].z;
        b += (size_t)n * (4 + 1 + 3 * sizeof(mgv)) + 5 * 256;
    }
    int64_t nc = (int64_t)dims.back().x * dims.back().y * dims.back().z;
    if (nc <= kCoarseMax) b += (size_t)nc * nc * 4 + 256;
    return b;
}

__device__ inline double hedge(int i, int n) { return (i == 0 || i == n - 1) ? 0.5 : 1.0; }

// ---------------------------------------------------------------------------
// Interpolation weights

// Along one axis, fine index f of a level with nc coarse nodes: its own
// coarse node c0 = f / 2 with weight w0 and the neighbour on its side c1
// (f even: c0 - 1, f odd: c0 + 1) with weight w1; without that neighbour
// w0 = 1, w1 = 0 and c1 = c0.
struct Interp1 {
    int c0, c1;
    double w0, w1;
};

__host__ __device__ inline Interp1 interp1(int f, int nc) {
    const int own = f >> 1, o = (f & 1) ? own + 1 : own - 1;
    const bool ok = o >= 0 && o < nc;
    Interp1 r;
    r.c0 = own;
    r.c1 = ok ? o : own;
    r.w0 = ok ? 0.75 : 1.0;
    r.w1 = ok ? 0.25 : 0.0;
    return r;
}

// Weight of coarse node J in the interpolation of fine index f (one axis).
__host__ __device__ inline double interp_w(int f, int J, int nc) {
    const Interp1 r = interp1(f, nc);
    return (r.c0 == J ? r.w0 : 0.0) + (r.c1 == J && r.c1 != r.c0 ? r.w1 : 0.0);
}

__device__ inline int clampi(int v, int n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }

// ---------------------------------------------------------------------------
// Set-up: unknowns and Galerkin rows

// used[J] = 1 when one of the 2x2x2 fine nodes of J is an unknown (finest:
// free node; coarser: used).
template <bool FINEST>
__global__ void k_mg_used(int fnx, int fny, int fnz, const uint8_t* __restrict__ fmask, MgLevel C) {
    int64_t J = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (J >= C.n) return;
    const int Jx = (int)(J % C.nx), Jy = (int)((J / C.nx) % C.ny), Jz = (int)(J / ((int64_t)C.nx * C.ny));
    uint8_t u = 0;
    for (int t = 0; t < 8; ++t) {
        int i = 2 * Jx + (t & 1), j = 2 * Jy + ((t >> 1) & 1), k = 2 * Jz + ((t >> 2) & 1);
        if (i >= fnx || j >= fny || k >= fnz) continue;
        uint8_t v = fmask[((int64_t)k * fny + j) * fnx + i];
        if (FINEST ? v == 0 : v != 0) u = 1;
    }
    C.used[J] = u;
}

// Row J of P^T A P: for every unknown fine node i interpolated from J (the
// 4x4x4 fine nodes 2J-1 .. 2J+2), P[i][J] times row i of A times P, the
// products added to the coarse offsets K - J in [-2, 2]^3. One thread per
// coarse node, its 125 accumulators in LDS (FP64), every row summed in the
// same order, so nodes with identical surroundings get identical rows.
constexpr int kGalBlock = 64;

struct GalerkinFine {  // row i of the finest operator, matrix-free from the node types
    Grid g;
    const uint8_t* type;
};

struct GalerkinCoarse {  // row i of a coarse operator from its class table
    MgLevel F;
};

template <typename SRC>
__device__ inline void galerkin_row(const SRC& src, const MgLevel& C, int64_t J, double* acc);

// scatter v (an entry of A P's column space at fine node (ii, jj, kk)) into
// the accumulators of coarse row J through the interpolation of that node
__device__ inline void gal_scatter(const MgLevel& C, int fnx, int fny, int fnz, int Jx, int Jy, int Jz, int ii, int jj,
                                   int kk, double v, double* acc) {
    (void)fnx;
    (void)fny;
    (void)fnz;
    const Interp1 px = interp1(ii, C.nx), py = interp1(jj, C.ny), pz = interp1(kk, C.nz);
    const int cx[2] = {px.c0, px.c1}, cy[2] = {py.c0, py.c1}, cz[2] = {pz.c0, pz.c1};
    const double wx[2] = {px.w0, px.w1}, wy[2] = {py.w0, py.w1}, wz[2] = {pz.w0, pz.w1};
    for (int a = 0; a < 2; ++a) {
        if (wz[a] == 0.0) continue;
        const int dz = cz[a] - Jz;
        for (int b = 0; b < 2; ++b) {
            if (wy[b] == 0.0) continue;
            const int dy = cy[b] - Jy;
            for (int c = 0; c < 2; ++c) {
                if (wx[c] == 0.0) continue;
                const int dx = cx[c] - Jx;
                if (dx < -2 || dx > 2 || dy < -2 || dy > 2 || dz < -2 || dz > 2) continue;  // not reached
                const int64_t K = ((int64_t)cz[a] * C.ny + cy[b]) * C.nx + cx[c];
                if (!C.used[K]) continue;
                acc[(25 * (dz + 2) + 5 * (dy + 2) + dx + 2) * kGalBlock] += v * (wz[a] * wy[b] * wx[c]);
            }
        }
    }
}

template <>
__device__ inline void galerkin_row<GalerkinFine>(const GalerkinFine& src, const MgLevel& C, int64_t J, double* acc) {
    const Grid& g = src.g;
    const int Jx = (int)(J % C.nx), Jy = (int)((J / C.nx) % C.ny), Jz = (int)(J / ((int64_t)C.nx * C.ny));
    for (int dk = -1; dk <= 2; ++dk) {
        const int k = 2 * Jz + dk;
        if (k < 0 || k >= g.nz) continue;
        const double pz = interp_w(k, Jz, C.nz);
        if (pz == 0.0) continue;
        for (int dj = -1; dj <= 2; ++dj) {
            const int j = 2 * Jy + dj;
            if (j < 0 || j >= g.ny) continue;
            const double py = interp_w(j, Jy, C.ny);
            if (py == 0.0) continue;
            for (int di = -1; di <= 2; ++di) {
                const int i = 2 * Jx + di;
                if (i < 0 || i >= g.nx) continue;
                const double px = interp_w(i, Jx, C.nx);
                if (px == 0.0) continue;
                const int64_t n = ((int64_t)k * g.ny + j) * g.nx + i;
                if (src.type[n] != 0) continue;
                const double wi = px * py * pz;
                const double fx = hedge(j, g.ny) * hedge(k, g.nz), fy = hedge(i, g.nx) * hedge(k, g.nz),
                             fz = hedge(i, g.nx) * hedge(j, g.ny);
                const int nbi[6] = {i - 1, i + 1, i, i, i, i}, nbj[6] = {j, j, j - 1, j + 1, j, j},
                          nbk[6] = {k, k, k, k, k - 1, k + 1};
                const double f[6] = {fx, fx, fy, fy, fz, fz};
                double dg = 0.0;
                for (int d = 0; d < 6; ++d) {
                    const int ii = nbi[d], jj = nbj[d], kk = nbk[d];
                    if (ii < 0 || ii >= g.nx || jj < 0 || jj >= g.ny || kk < 0 || kk >= g.nz) continue;
                    dg += f[d];
                }
                gal_scatter(C, g.nx, g.ny, g.nz, Jx, Jy, Jz, i, j, k, wi * dg, acc);
                for (int d = 0; d < 6; ++d) {
                    const int ii = nbi[d], jj = nbj[d], kk = nbk[d];
                    if (ii < 0 || ii >= g.nx || jj < 0 || jj >= g.ny || kk < 0 || kk >= g.nz) continue;
                    if (src.type[((int64_t)kk * g.ny + jj) * g.nx + ii] != 0) continue;
                    gal_scatter(C, g.nx, g.ny, g.nz, Jx, Jy, Jz, ii, jj, kk, -wi * f[d], acc);
                }
            }
        }
    }
}

template <>
__device__ inline void galerkin_row<GalerkinCoarse>(const GalerkinCoarse& src, const MgLevel& C, int64_t J,
                                                    double* acc) {
    const MgLevel& F = src.F;
    const int Jx = (int)(J % C.nx), Jy = (int)((J / C.nx) % C.ny), Jz = (int)(J / ((int64_t)C.nx * C.ny));
    for (int dk = -1; dk <= 2; ++dk) {
        const int k = 2 * Jz + dk;
        if (k < 0 || k >= F.nz) continue;
        const double pz = interp_w(k, Jz, C.nz);
        if (pz == 0.0) continue;
        for (int dj = -1; dj <= 2; ++dj) {
            const int j = 2 * Jy + dj;
            if (j < 0 || j >= F.ny) continue;
            const double py = interp_w(j, Jy, C.ny);
            if (py == 0.0) continue;
            for (int di = -1; di <= 2; ++di) {
                const int i = 2 * Jx + di;
                if (i < 0 || i >= F.nx) continue;
                const double px = interp_w(i, Jx, C.nx);
                if (px == 0.0) continue;
                const int64_t n = ((int64_t)k * F.ny + j) * F.nx + i;
                const uint32_t cls = F.id[n];
                if (cls == 0) continue;
                const double wi = px * py * pz;
                const float* row = F.tab + (size_t)cls * kTabRow;
                for (int o = 0; o < 125; ++o) {
                    const double a = row[o];
                    if (a == 0.0) continue;
                    const int ii = i + o % 5 - 2, jj = j + (o / 5) % 5 - 2, kk = k + o / 25 - 2;
                    if (ii < 0 || ii >= F.nx || jj < 0 || jj >= F.ny || kk < 0 || kk >= F.nz) continue;  // not stored
                    gal_scatter(C, F.nx, F.ny, F.nz, Jx, Jy, Jz, ii, jj, kk, wi * a, acc);
                }
            }
        }
    }
}

template <typename SRC>
__global__ __launch_bounds__(kGalBlock) void k_mg_galerkin(SRC src, MgLevel C, float* __restrict__ rows) {
    __shared__ double acc[125 * kGalBlock];
    const int t = threadIdx.x;
    const int64_t J = (int64_t)blockIdx.x * kGalBlock + t;
    for (int o = 0; o < 125; ++o) acc[o * kGalBlock + t] = 0.0;
    if (J < C.n && C.used[J]) galerkin_row<SRC>(src, C, J, acc + t);
    if (J < C.n)
        for (int o = 0; o < 125; ++o) rows[J * 125 + o] = (float)acc[o * kGalBlock + t];
}

struct MgArgs {
    Grid g;
    const uint8_t* type;
    DevState* s;
    double* part_rr;   // CG partials of r.r (finest level, read by the first kernel)
    double* part_bb;   // CG partials of b.b (read before the first iteration)
    double* part_rz;   // partials of r.z written by the last kernel
    int cg_blocks;     // number of CG partials
};

// Convergence test of the CG update, taken by every block of the first
// kernel of the V-cycle: finishes r.r (and b.b before the first iteration)
// from the CG partials in a fixed order, so every block gets the same
// answer; block 0 stores it (and sets done on convergence). All threads of
// the block must call it.
__device__ inline bool mg_test(const MgArgs& a) {
    DevState* s = a.s;
    const double rr = sum_partials_n(a.part_rr, a.cg_blocks);
    const bool first = s->it == 0;
    const double bb = first ? sum_partials_n(a.part_bb, a.cg_blocks) : s->bb;
    const bool conv = (bb == 0.0) || (sqrt(rr) <= s->rtol * sqrt(bb)) || (s->it >= s->maxit);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (first) {
            s->bb = bb;
            s->rr0 = rr;
        }
        s->rr = rr;
        if (conv) {
            s->done = 1;
            s->zero_solution = (bb == 0.0);
        }
    }
    return conv;
}

// Coarse-level kernels run on a grid of (plane tiles, planes): a block is a
// tile of kBlock nodes of one plane (32-bit in-plane indices). The linear
// block index is remapped so that consecutive planes run on one XCD and the
// planes a stencil or a transfer shares stay in that XCD's L2.
struct PlaneIdx {
    int i, j, k, p;
    int64_t n;
};

__device__ inline void plane_block(int& bx, int& bz) {
    const uint32_t nbx = gridDim.x;
    const uint32_t b = (uint32_t)xcd_block((int64_t)blockIdx.y * nbx + blockIdx.x, (int64_t)nbx * gridDim.y);
    bz = (int)(b / nbx);
    bx = (int)(b - (uint32_t)bz * nbx);
}

__device__ inline bool plane_idx(int nx, int ny, PlaneIdx& q) {
    const int pl = nx * ny;
    int bx, bz;
    plane_block(bx, bz);
    q.p = bx * kBlock + (int)threadIdx.x;
    if (q.p >= pl) return false;
    q.k = bz;
    q.j = q.p / nx;
    q.i = q.p - q.j * nx;
    q.n = (int64_t)q.k * pl + q.p;
    return true;
}

// (row . x) at node (i, j, k) of a coarse level for the class row t
// (coefficient index 25 (dz + 2) + 5 (dy + 2) + dx + 2), as
// sum_o t_o (x_o - x_c) + (sum_o t_o) x_c: the differences of neighbouring
// values are small where x is smooth, so the 125 products are accumulated in
// FP32 without the cancellation of a plain sum; the row-sum term is FP64.
// Offsets outside the grid have zero coefficients and are read at the
// clamped position, so every load is unconditional (32-bit byte offsets from
// the level's base pointer; a coarse level is far below 4 GiB).
__device__ inline double row_dot(const MgLevel& L, const mgv* __restrict__ x, int i, int j, int k, float xc,
                                 const float* __restrict__ t) {
    uint32_t xs[5], rows[25];
    const uint32_t pl = (uint32_t)(L.nx * L.ny);
#pragma unroll
    for (int d = 0; d < 5; ++d) xs[d] = 4u * (uint32_t)clampi(i + d - 2, L.nx);
#pragma unroll
    for (int dz = 0; dz < 5; ++dz) {
        const uint32_t zr = (uint32_t)clampi(k + dz - 2, L.nz) * pl;
#pragma unroll
        for (int dy = 0; dy < 5; ++dy) rows[5 * dz + dy] = 4u * (zr + (uint32_t)(clampi(j + dy - 2, L.ny) * L.nx));
    }
    const char* __restrict__ xb = (const char*)x;
    float s = 0.0f;
#pragma unroll
    for (int r = 0; r < 25; ++r) {
#pragma unroll
        for (int dx = 0; dx < 5; ++dx) s = fmaf(t[5 * r + dx], *(const float*)(xb + (rows[r] + xs[dx])) - xc, s);
    }
    return (double)s + (double)t[kTabSum] * (double)xc;
}

// One damped Jacobi sweep on a coarse level, xo = xi + omega D^-1 (b - A xi);
// with RESID the residual b - A xi instead (zero where there is no unknown).
// A wavefront covers a run of nodes of one plane, which holds only a few row
// classes (the interior one and those of the faces it touches): the
// wavefront copies each distinct row once into LDS (up to kSlots rows; the
// slot stride is odd, so lanes of different slots read different banks) and
// the lanes read their coefficients there. A wavefront with more classes
// (near the tip) reads the rows from the table per lane.
constexpr int kSlots = 8, kSlotStride = 129;

template <bool RESID>
__global__ __launch_bounds__(kBlock) void k_mg_sweep(MgArgs a, MgLevel L, const float* __restrict__ tab,
                                                      const mgv* __restrict__ xi, mgv* __restrict__ xo) {
    __shared__ float slots[kBlock / 64][kSlots * kSlotStride];
    PlaneIdx q;
    const bool in = plane_idx(L.nx, L.ny, q);
    if (!in) {  // lanes past the plane work on its last node and store nothing
        q.p = L.nx * L.ny - 1;
        q.j = L.ny - 1;
        q.i = L.nx - 1;
        q.n = (int64_t)q.k * L.nx * L.ny + q.p;
    }
    const uint32_t cls = L.id[q.n];
    const double bn = L.b[q.n];
    const float xn = xi[q.n];
    if (a.s->done) return;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float* sw = slots[w];
    // distinct classes of the wavefront, in order of their first lane
    int slot = -1, ns = 0;
    unsigned long long rem = __ballot(true);
    while (rem && ns < kSlots) {
        const int lead = __ffsll((long long)rem) - 1;
        const uint32_t c = __shfl(cls, lead);
        const unsigned long long m = __ballot(cls == c);
        if (cls == c) slot = ns;
        const float* src = tab + (size_t)c * kTabRow;
        sw[ns * kSlotStride + lane] = src[lane];
        sw[ns * kSlotStride + 64 + lane] = src[64 + lane];
        rem &= ~m;
        ++ns;
    }
    __builtin_amdgcn_wave_barrier();
    double ax;
    float invd;
    if (rem == 0) {
        const float* t = sw + slot * kSlotStride;
        ax = row_dot(L, xi, q.i, q.j, q.k, xn, t);
        invd = t[kTabInvD];
    } else {
        const float* t = tab + (size_t)cls * kTabRow;
        ax = row_dot(L, xi, q.i, q.j, q.k, xn, t);
        invd = t[kTabInvD];
    }
    if (!in) return;
    if (RESID)
        xo[q.n] = (mgv)((bn - ax) * (double)(cls != 0));
    else
        xo[q.n] = (mgv)((double)xn + (double)invd * (bn - ax));  // class 0: xn = 0, omega / D = 0
}

// The same sweep on a large coarse level as a z-marching kernel: a block is
// a 16 x 16 (x, y) tile of columns walking kc planes, each wavefront an 8 x 8
// patch of it. Each plane of xi is staged once in LDS with a halo of two
// nodes (20 x 20 values, clamped at the grid faces where the coefficients are
// zero) in a ring of six planes. A patch away from the faces and the tip
// holds one row class: its coefficients are then wave-uniform (scalar
// loads); other patches keep their classes in LDS slots as above, refreshed
// when a plane brings another set of classes. One barrier per plane: step k
// loads plane k + 2 into the slot of plane k - 4, which no thread reads after
// step k - 2.
// An LDS plane holds kZH rows of kZH values at a row pitch of kZP floats:
// with the pitch 24 the 8 rows of an 8 x 8 patch fall into distinct banks.
constexpr int kZT = 16, kZH = kZT + 4, kZP = 24, kZRing = 6, kZHalo = kZH * kZH, kZPlane = kZH * kZP;

__device__ inline int zring(int k) { return (k + 2 * kZRing) % kZRing; }  // k >= -2

inline unsigned zgrid16(int nx, int ny, int nz, int target, int* kc) {
    const int64_t cols = (int64_t)((nx + kZT - 1) / kZT) * ((ny + kZT - 1) / kZT);
    int64_t k = (nz * cols + target - 1) / target;
    if (k < 1) k = 1;
    *kc = (int)k;
    return (unsigned)(cols * ((nz + k - 1) / k));
}

// sum_o t_o (x_o - x_c) + (sum_o t_o) x_c from the staged planes; lb is the
// offset of the node's 5 x 5 window (its corner) in a plane
__device__ inline double ring_dot(const float (*sx)[kZPlane], int k, int lb, float xc, const float* __restrict__ t) {
    float s = 0.0f;
#pragma unroll
    for (int dz = 0; dz < 5; ++dz) {
        // one address per plane, the 25 reads at constant offsets from it
        // (the empty asm keeps the compiler from hoisting 25 per-lane
        // addresses out of the loop and adding the plane base to each)
        int a = lb;
        asm volatile("" : "+v"(a));
        const float* pln = sx[zring(k + dz - 2)] + a;
        float c[25], v[25];
#pragma unroll
        for (int q = 0; q < 25; ++q) c[q] = t[25 * dz + q];
#pragma unroll
        for (int q = 0; q < 25; ++q) v[q] = pln[(q / 5) * kZP + q % 5];
#pragma unroll
        for (int q = 0; q < 25; ++q) s = fmaf(c[q], v[q] - xc, s);
    }
    return (double)s + (double)t[kTabSum] * (double)xc;
}

template <bool RESID>
__global__ __launch_bounds__(kBlock) void k_mg_sweep_z(MgArgs a, MgLevel L, const float* __restrict__ tab,
                                                        const mgv* __restrict__ xi, mgv* __restrict__ xo, int kc) {
    // one LDS array, the plane ring first: a plane's 25 reads then fit in the
    // offset fields of the read instructions from one address
    __shared__ float lds[kZRing * kZPlane + (kBlock / 64) * kSlots * kSlotStride];
    float(*sx)[kZPlane] = (float(*)[kZPlane])lds;
    if (a.s->done) return;  // the same for every thread of the block
    const int ntx = (L.nx + kZT - 1) / kZT, nty = (L.ny + kZT - 1) / kZT;
    const int64_t b = xcd_block(blockIdx.x, gridDim.x);
    const int bx = (int)(b % ntx);
    const int64_t rb = b / ntx;
    const int by = (int)(rb % nty), bz = (int)(rb / nty);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tx = 8 * (w & 1) + (lane & 7), ty = 8 * (w >> 1) + (lane >> 3);  // position in the tile
    const int x0 = bx * kZT, y0 = by * kZT;
    const int i = x0 + tx, j = y0 + ty;
    const bool col = i < L.nx && j < L.ny;
    const int k0 = bz * kc, k1 = k0 + kc < L.nz ? k0 + kc : L.nz;
    const int pl = L.nx * L.ny;
    // halo values loaded by this thread: e = threadIdx.x + 256 q, e < 400
    int off[2], doff[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int e = (int)threadIdx.x + kBlock * q;
        const int ee = e < kZHalo ? e : 0;
        const int hy = ee / kZH, hx = ee - hy * kZH;
        off[q] = clampi(y0 - 2 + hy, L.ny) * L.nx + clampi(x0 - 2 + hx, L.nx);
        doff[q] = hy * kZP + hx;
    }
    const bool second = (int)threadIdx.x + kBlock < kZHalo;
    // plane kk (clamped into the grid) into registers, and from there into
    // its ring slot
    auto fetch = [&](int kk, float& v0, float& v1) {
        const mgv* src = xi + (int64_t)clampi(kk, L.nz) * pl;
        v0 = src[off[0]];
        v1 = src[second ? off[1] : off[0]];
    };
    auto put = [&](int kk, float v0, float v1) {
        float* dst = sx[zring(kk)];
        dst[doff[0]] = v0;
        if (second) dst[doff[1]] = v1;
    };
    const int ic = i < L.nx ? i : L.nx - 1, jc = j < L.ny ? j : L.ny - 1;
    const int64_t n0 = (int64_t)k0 * pl + jc * L.nx + ic;
    // Every value a step needs is loaded during the step before it: plane
    // k + 2 of the ring, the class id and b of node k. The first planes and
    // step are all issued before the first wait.
    float pro[4][2];
#pragma unroll
    for (int q = 0; q < 4; ++q) fetch(k0 - 2 + q, pro[q][0], pro[q][1]);
    float pv0, pv1;
    fetch(k0 + 2, pv0, pv1);
    uint32_t cls_next = L.id[n0];
    float b_next = L.b[n0];
#pragma unroll
    for (int q = 0; q < 4; ++q) put(k0 - 2 + q, pro[q][0], pro[q][1]);
    const int hx = tx + 2, hy = ty + 2;
    const int lb = (hy - 2) * kZP + hx - 2;  // the node's 5 x 5 window in a plane
    float* sw = lds + kZRing * kZPlane + w * (kSlots * kSlotStride);
    int slot = -1;
    bool staged = false;  // the patch's classes are all in its slots
    uint32_t prev = 0xFFFFFFFFu;
    for (int k = k0; k < k1; ++k) {
        put(k + 2, pv0, pv1);
        const int64_t n = (int64_t)k * pl + jc * L.nx + ic;
        const uint32_t cls = cls_next;
        const double bn = (double)b_next;
        // the next step's loads (at the last step, node k again)
        const int64_t nn = k + 1 < k1 ? n + pl : n;
        fetch(k + 3, pv0, pv1);
        cls_next = L.id[nn];
        b_next = L.b[nn];
        __syncthreads();
        const float xn = sx[zring(k)][hy * kZP + hx];
        const uint32_t c0 = __builtin_amdgcn_readfirstlane(cls);
        double ax;
        float invd;
        if (__all(cls == c0)) {
            const float* tt = tab + (size_t)c0 * kTabRow;
            ax = ring_dot(sx, k, lb, xn, tt);
            invd = tt[kTabInvD];
        } else {
            if (!__all(cls == prev)) {
                slot = -1;
                int ns = 0;
                unsigned long long rem = __ballot(true);
                while (rem && ns < kSlots) {
                    const int lead = __ffsll((long long)rem) - 1;
                    const uint32_t c = __shfl(cls, lead);
                    const unsigned long long m = __ballot(cls == c);
                    if (cls == c) slot = ns;
                    const float* src = tab + (size_t)c * kTabRow;
                    sw[ns * kSlotStride + lane] = src[lane];
                    sw[ns * kSlotStride + 64 + lane] = src[64 + lane];
                    rem &= ~m;
                    ++ns;
                }
                staged = rem == 0;
                prev = cls;
                __builtin_amdgcn_wave_barrier();
            }
            if (staged) {
                const float* tt = sw + slot * kSlotStride;
                ax = ring_dot(sx, k, lb, xn, tt);
                invd = tt[kTabInvD];
            } else {
                const float* tt = tab + (size_t)cls * kTabRow;
                ax = ring_dot(sx, k, lb, xn, tt);
                invd = tt[kTabInvD];
            }
        }
        const mgv out = RESID ? (mgv)((bn - ax) * (double)(cls != 0)) : (mgv)((double)xn + (double)invd * (bn - ax));
        if (col) xo[n] = out;
    }
}

// Stores the restricted residual b of coarse node n and, when first is set,
// also the first pre-smoothing sweep from x = 0, x = omega D^-1 b (from the
// FP32 value of b; zero where there is no unknown, whose table row holds
// omega / D = 0).
__device__ inline void store_restricted(const MgLevel& C, int64_t n, double s, int first) {
    const mgv bn = (mgv)s;
    C.b[n] = bn;
    if (first) C.x0[n] = (mgv)((double)C.tab[(size_t)C.id[n] * kTabRow + kTabInvD] * (double)bn);
}

// b_c = P^T r for an even fine width (fnx = 2 C.nx): each lane reads its
// two fine nodes 2J, 2J+1 of a row as one float2 and 2J-1, 2J+2 as single
// values (clamped at the row ends, where their weight is zero); every load is
// unconditional, so all 48 are in flight together. Row sums in FP32 (weights
// 1/4, 3/4, 1), the y and z sums in FP64.
__global__ __launch_bounds__(kBlock) void k_mg_restrict2(MgArgs a, int fnx, int fny, int fnz, const mgv* __restrict__ r,
                                                          MgLevel C, int first) {
    PlaneIdx q;
    if (!plane_idx(C.nx, C.ny, q)) return;
    const int Jx = q.i, Jy = q.j, Jz = q.k;
    float wx[4];
    double wy[4], wz[4];
    uint32_t rowo[16];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const int fi = 2 * Jx - 1 + d, fj = 2 * Jy - 1 + d, fk = 2 * Jz - 1 + d;
        wx[d] = (fi >= 0 && fi < fnx) ? (float)interp_w(fi, Jx, C.nx) : 0.0f;
        wy[d] = (fj >= 0 && fj < fny) ? interp_w(fj, Jy, C.ny) : 0.0;
        wz[d] = (fk >= 0 && fk < fnz) ? interp_w(fk, Jz, C.nz) : 0.0;
    }
#pragma unroll
    for (int dz = 0; dz < 4; ++dz)
#pragma unroll
        for (int dy = 0; dy < 4; ++dy)
            rowo[4 * dz + dy] = (uint32_t)clampi(2 * Jz - 1 + dz, fnz) * (uint32_t)(fnx * fny) +
                                (uint32_t)(clampi(2 * Jy - 1 + dy, fny) * fnx);
    const uint32_t il = (uint32_t)clampi(2 * Jx - 1, fnx), ip = (uint32_t)(2 * Jx), ir = (uint32_t)clampi(2 * Jx + 2, fnx);
    float lv[16], rv[16];
    float2 pv[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        lv[e] = r[rowo[e] + il];
        pv[e] = *(const float2*)(r + rowo[e] + ip);
        rv[e] = r[rowo[e] + ir];
    }
    double s = 0.0;
#pragma unroll
    for (int dz = 0; dz < 4; ++dz) {
        double sy = 0.0;
#pragma unroll
        for (int dy = 0; dy < 4; ++dy) {
            const int e = 4 * dz + dy;
            float sx = wx[0] * lv[e];
            sx = fmaf(wx[1], pv[e].x, sx);
            sx = fmaf(wx[2], pv[e].y, sx);
            sx = fmaf(wx[3], rv[e], sx);
            sy += wy[dy] * (double)sx;
        }
        s += wz[dz] * sy;
    }
    const uint8_t u = C.used[q.n];
    if (a.s->done) return;
    store_restricted(C, q.n, s * (double)u, first);
}

// k_mg_restrict2 marching in z: a thread takes one coarse column over kc
// coarse planes. Coarse planes Jz and Jz + 1 share the fine planes 2Jz + 1
// and 2Jz + 2, so a step reads two new fine planes (four rows of four nodes
// each) and keeps the x-y sums of the other two; the sums and their order
// are those of k_mg_restrict2, so the results agree bit for bit.
__global__ __launch_bounds__(kBlock) void k_mg_restrict2z(MgArgs a, int fnx, int fny, int fnz,
                                                           const mgv* __restrict__ r, MgLevel C, int first, int kc) {
    if (a.s->done) return;
    const ZMarch t = zmarch(C.nx, C.ny, C.nz, kc);
    if (!t.col) return;
    const int Jx = t.i, Jy = t.j;
    float wx[4];
    double wy[4];
    uint32_t rowo[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const int fi = 2 * Jx - 1 + d, fj = 2 * Jy - 1 + d;
        wx[d] = (fi >= 0 && fi < fnx) ? (float)interp_w(fi, Jx, C.nx) : 0.0f;
        wy[d] = (fj >= 0 && fj < fny) ? interp_w(fj, Jy, C.ny) : 0.0;
        rowo[d] = (uint32_t)(clampi(fj, fny) * fnx);
    }
    const uint32_t il = (uint32_t)clampi(2 * Jx - 1, fnx), ip = (uint32_t)(2 * Jx), ir = (uint32_t)clampi(2 * Jx + 2, fnx);
    const uint32_t fpl = (uint32_t)(fnx * fny);
    // the 16 values of fine plane fk a coarse node takes (clamped; the z
    // weight of a plane outside the grid is zero), and their x-y sum
    struct Pl {
        float l[4], r[4];
        float2 p[4];
    };
    auto load = [&](int fk, Pl& v) {
        const uint32_t o = (uint32_t)clampi(fk, fnz) * fpl;
#pragma unroll
        for (int dy = 0; dy < 4; ++dy) {
            v.l[dy] = r[o + rowo[dy] + il];
            v.p[dy] = *(const float2*)(r + o + rowo[dy] + ip);
            v.r[dy] = r[o + rowo[dy] + ir];
        }
    };
    auto xysum = [&](const Pl& v) -> double {
        double sy = 0.0;
#pragma unroll
        for (int dy = 0; dy < 4; ++dy) {
            float sx = wx[0] * v.l[dy];
            sx = fmaf(wx[1], v.p[dy].x, sx);
            sx = fmaf(wx[2], v.p[dy].y, sx);
            sx = fmaf(wx[3], v.r[dy], sx);
            sy += wy[dy] * (double)sx;
        }
        return sy;
    };
    // the two new planes of a step are loaded one step ahead
    Pl a2, a3;
    double s0, s1;
    {
        Pl a0, a1;
        load(2 * t.k0 - 1, a0);
        load(2 * t.k0, a1);
        load(2 * t.k0 + 1, a2);
        load(2 * t.k0 + 2, a3);
        s0 = xysum(a0);
        s1 = xysum(a1);
    }
    const int64_t cpl = (int64_t)C.nx * C.ny;
    int64_t n = (int64_t)t.k0 * cpl + (int64_t)Jy * C.nx + Jx;
    for (int Jz = t.k0; Jz < t.k1; ++Jz, n += cpl) {
        const double s2 = xysum(a2), s3 = xysum(a3);
        if (Jz + 1 < t.k1) {
            load(2 * Jz + 3, a2);
            load(2 * Jz + 4, a3);
        }
        double wz[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const int fk = 2 * Jz - 1 + d;
            wz[d] = (fk >= 0 && fk < fnz) ? interp_w(fk, Jz, C.nz) : 0.0;
        }
        double sum = 0.0;
        sum += wz[0] * s0;
        sum += wz[1] * s1;
        sum += wz[2] * s2;
        sum += wz[3] * s3;
        store_restricted(C, n, sum * (double)C.used[n], first);
        s0 = s2;
        s1 = s3;
    }
}

// b_c = P^T r: coarse node J collects the fine nodes 2J-1 .. 2J+2 of each
// axis with their interpolation weights (zero where J is not an unknown).
__global__ __launch_bounds__(kBlock) void k_mg_restrict(MgArgs a, int fnx, int fny, int fnz, const mgv* __restrict__ r,
                                                         MgLevel C, int first) {
    PlaneIdx q;
    if (!plane_idx(C.nx, C.ny, q)) return;
    const int Jx = q.i, Jy = q.j, Jz = q.k;
    double wx[4], wy[4], wz[4];
    int ix[4], jy[4];
    int64_t kz[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const int fi = 2 * Jx - 1 + d, fj = 2 * Jy - 1 + d, fk = 2 * Jz - 1 + d;
        wx[d] = (fi >= 0 && fi < fnx) ? interp_w(fi, Jx, C.nx) : 0.0;
        wy[d] = (fj >= 0 && fj < fny) ? interp_w(fj, Jy, C.ny) : 0.0;
        wz[d] = (fk >= 0 && fk < fnz) ? interp_w(fk, Jz, C.nz) : 0.0;
        ix[d] = clampi(fi, fnx);
        jy[d] = clampi(fj, fny) * fnx;
        kz[d] = (int64_t)clampi(fk, fnz) * fnx * fny;
    }
    const uint8_t u = C.used[q.n];
    double s = 0.0;
#pragma unroll
    for (int dz = 0; dz < 4; ++dz) {
        double sy = 0.0;
#pragma unroll
        for (int dy = 0; dy < 4; ++dy) {
            const mgv* row = r + kz[dz] + jy[dy];
            double sx = 0.0;
#pragma unroll
            for (int dx = 0; dx < 4; ++dx) sx += wx[dx] * (double)row[ix[dx]];
            sy += wy[dy] * sx;
        }
        s += wz[dz] * sy;
    }
    if (a.s->done) return;
    store_restricted(C, q.n, s * (double)u, first);
}

// xo = xi + P xc on a level of fnx x fny x fnz nodes (zero where the node is
// not an unknown: finest level, type != 0; coarser, used == 0). xc is zero on
// coarse nodes without an unknown, which drops P's columns for them.
template <bool FINEST>
__global__ __launch_bounds__(kBlock) void k_mg_prolong(MgArgs a, int fnx, int fny, int fnz,
                                                        const uint8_t* __restrict__ fmask, const mgv* __restrict__ xi,
                                                        mgv* __restrict__ xo, MgLevel C, const mgv* __restrict__ xc) {
    (void)fnz;
    PlaneIdx q;
    if (!plane_idx(fnx, fny, q)) return;
    const Interp1 px = interp1(q.i, C.nx), py = interp1(q.j, C.ny), pz = interp1(q.k, C.nz);
    const int cpl = C.nx * C.ny;
    const int64_t z0 = (int64_t)pz.c0 * cpl, z1 = (int64_t)pz.c1 * cpl;
    const int y0 = py.c0 * C.nx, y1 = py.c1 * C.nx;
    const double v000 = xc[z0 + y0 + px.c0], v001 = xc[z0 + y0 + px.c1], v010 = xc[z0 + y1 + px.c0],
                 v011 = xc[z0 + y1 + px.c1], v100 = xc[z1 + y0 + px.c0], v101 = xc[z1 + y0 + px.c1],
                 v110 = xc[z1 + y1 + px.c0], v111 = xc[z1 + y1 + px.c1];
    const uint8_t m = fmask[q.n];
    const double xv = xi[q.n];
    if (a.s->done) return;
    const double s0 = py.w0 * (px.w0 * v000 + px.w1 * v001) + py.w1 * (px.w0 * v010 + px.w1 * v011);
    const double s1 = py.w0 * (px.w0 * v100 + px.w1 * v101) + py.w1 * (px.w0 * v110 + px.w1 * v111);
    const bool unknown = FINEST ? m == 0 : m != 0;
    xo[q.n] = (mgv)((xv + pz.w0 * s0 + pz.w1 * s1) * (double)unknown);
}

// The finest-level prolongation for an even width, two x nodes 2m, 2m+1 per
// lane: both take 3/4 of coarse column m and 1/4 of m - 1 and m + 1
// respectively (all of m at the grid edges), so a lane reads three coarse
// values per (y, z) pair of coarse rows and stores a float2. FP32 arithmetic
// (the weights are exact).
__global__ __launch_bounds__(kBlock) void k_mg_prolong2(MgArgs a, int fnx, int fny, const uint8_t* __restrict__ type,
                                                         const mgv* __restrict__ xi, mgv* __restrict__ xo, MgLevel C,
                                                         const mgv* __restrict__ xc) {
    const int hx = fnx >> 1;  // lanes per row
    const int pl = hx * fny;
    int bx, k;
    plane_block(bx, k);
    const int p = bx * kBlock + (int)threadIdx.x;
    if (p >= pl) return;
    const int j = p / hx, m = p - j * hx;
    const int64_t n = (int64_t)k * fnx * fny + (int64_t)j * fnx + 2 * m;
    const Interp1 py = interp1(j, C.ny), pz = interp1(k, C.nz);
    const int mw = m > 0 ? m - 1 : m, me = m + 1 < C.nx ? m + 1 : m;
    const float a0 = m > 0 ? 0.75f : 1.0f, aw = m > 0 ? 0.25f : 0.0f;           // node 2m
    const float a1 = m + 1 < C.nx ? 0.75f : 1.0f, ae = m + 1 < C.nx ? 0.25f : 0.0f;  // node 2m + 1
    const int cpl = C.nx * C.ny;
    const int r00 = pz.c0 * cpl + py.c0 * C.nx, r01 = pz.c0 * cpl + py.c1 * C.nx;
    const int r10 = pz.c1 * cpl + py.c0 * C.nx, r11 = pz.c1 * cpl + py.c1 * C.nx;
    const float w00 = (float)(pz.w0 * py.w0), w01 = (float)(pz.w0 * py.w1), w10 = (float)(pz.w1 * py.w0),
                w11 = (float)(pz.w1 * py.w1);
    const float c00 = xc[r00 + m], w00v = xc[r00 + mw], e00 = xc[r00 + me];
    const float c01 = xc[r01 + m], w01v = xc[r01 + mw], e01 = xc[r01 + me];
    const float c10 = xc[r10 + m], w10v = xc[r10 + mw], e10 = xc[r10 + me];
    const float c11 = xc[r11 + m], w11v = xc[r11 + mw], e11 = xc[r11 + me];
    const float2 xv = *(const float2*)(xi + n);
    const uchar2 tv = *(const uchar2*)(type + n);
    if (a.s->done) return;
    // per coarse (y, z) row: the column sums for node 2m (west side) and 2m + 1 (east side)
    float s0 = 0.0f, s1 = 0.0f;
    s0 = fmaf(w00, fmaf(a0, c00, aw * w00v), s0);
    s1 = fmaf(w00, fmaf(a1, c00, ae * e00), s1);
    s0 = fmaf(w01, fmaf(a0, c01, aw * w01v), s0);
    s1 = fmaf(w01, fmaf(a1, c01, ae * e01), s1);
    s0 = fmaf(w10, fmaf(a0, c10, aw * w10v), s0);
    s1 = fmaf(w10, fmaf(a1, c10, ae * e10), s1);
    s0 = fmaf(w11, fmaf(a0, c11, aw * w11v), s0);
    s1 = fmaf(w11, fmaf(a1, c11, ae * e11), s1);
    float2 out;
    out.x = (xv.x + s0) * (float)(tv.x == 0);
    out.y = (xv.y + s1) * (float)(tv.y == 0);
    *(float2*)(xo + n) = out;
}

// Coarsest level: x = A^-1 b with the stored inverse, one wavefront per row
// (16-byte loads when the row length is a multiple of 4; rows and b start on
// 256-byte boundaries).
__global__ __launch_bounds__(kBlock) void k_mg_coarsest(MgArgs a, MgLevel L, const float* __restrict__ inv) {
    if (a.s->done) return;
    const int row = (int)(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int n = (int)L.n;
    if (row >= n) return;
    const float* r = inv + (size_t)row * n;
    double acc = 0.0;
    if ((n & 3) == 0) {
        const float4* r4 = (const float4*)r;
        const float4* b4 = (const float4*)L.b;
#pragma unroll 8
        for (int c = lane; c < (n >> 2); c += 64) {
            const float4 w = r4[c], v = b4[c];
            acc += (double)w.x * v.x + (double)w.y * v.y + (double)w.z * v.z + (double)w.w * v.w;
        }
    } else {
#pragma unroll 8
        for (int c = lane; c < n; c += 64) acc += (double)r[c] * (double)L.b[c];
    }
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

// Input value of a fine kernel at node m:
//   kFineFirst: the first sweep from zero, omega_1 b / D (b is zero on fixed nodes);
//   kFinePlain, kFineResid: xi (zero on fixed nodes).
// The diagonal of a free node does not depend on k (free nodes are never on
// a z face), so kFineFirst takes omega_1 / D of the node's column, cw.
constexpr int kFinePlain = 0, kFineFirst = 1, kFineResid = 3;

template <int MODE, typename TB>
struct FineIn {
    const mgv* __restrict__ xi;
    const TB* __restrict__ b;
    __device__ double operator()(int64_t m, double cw) const {
        if (MODE == kFineFirst) return cw * (double)b[m];
        return (double)xi[m];
    }
};

// omega / D for a free node of column (i, j) (zero outside the grid)
__device__ inline double col_weight(const Grid& g, int i, int j, double omega) {
    if (i < 0 || i >= g.nx || j < 0 || j >= g.ny) return 0.0;
    return omega / fine_diag(g, i, j, 1 < g.nz - 1 ? 1 : 0);
}

// One damped Jacobi sweep on the finest level with the weight w_out
// (kFineFirst: the convergence test of the CG update, then two sweeps from
// zero, the first with the weight w_in; kFineResid: the residual b - A xi
// instead); with LAST the partials of r.z (b . xo) are written, one per
// block.
template <int MODE, bool LAST, typename TB>
__global__ __launch_bounds__(kBlock) void k_mg_fine_sweep(MgArgs a, const TB* __restrict__ b0, const mgv* __restrict__ xi,
                                                           mgv* __restrict__ xo, int kc, double w_out, double w_in) {
    DevState* s = a.s;
    if (s->done) return;
    if (MODE == kFineFirst && mg_test(a)) return;
    const Grid& g = a.g;
    FineIn<MODE, TB> in{xi, b0};
    ZMarch t = zmarch(g.nx, g.ny, g.nz, kc);
    double rz = 0.0;
    if (t.col) {
        int i = t.i, j = t.j;
        int64_t pl = (int64_t)g.nx * g.ny;
        int64_t n = (int64_t)t.k0 * pl + (int64_t)j * g.nx + i;
        double hx = hedge(i, g.nx), hy = hedge(j, g.ny), fz = hx * hy;
        const double cwo = col_weight(g, i, j, w_out);
        double cw = 0.0, cwW = 0.0, cwE = 0.0, cwS = 0.0, cwN = 0.0;
        if (MODE == kFineFirst) {
            cw = col_weight(g, i, j, w_in);
            cwW = col_weight(g, i - 1, j, w_in);
            cwE = col_weight(g, i + 1, j, w_in);
            cwS = col_weight(g, i, j - 1, w_in);
            cwN = col_weight(g, i, j + 1, w_in);
        }
        // neighbours outside the grid are read at the node itself (every load
        // is unconditional, so a step's loads are issued together) and given
        // a zero weight
        const int iw = i > 0 ? i - 1 : i, ie = i < g.nx - 1 ? i + 1 : i;
        const int js = j > 0 ? j - 1 : j, jn = j < g.ny - 1 ? j + 1 : j;
        const int64_t ow = iw - i, oe = ie - i, os = (int64_t)(js - j) * g.nx, on = (int64_t)(jn - j) * g.nx;
        const double ww = i > 0 ? hy : 0.0, we = i < g.nx - 1 ? hy : 0.0;
        const double ws = j > 0 ? hx : 0.0, wn = j < g.ny - 1 ? hx : 0.0;
        double vm = in(t.k0 > 0 ? n - pl : n, cw);
        if (t.k0 == 0) vm = 0.0;
        double vc = in(n, cw);
        // kFineFirst: b of the node, carried from the previous step's load of
        // the plane above (a load of b0[n] of its own came after the waits
        // for the neighbours, a second memory latency per step)
        double bc = MODE == kFineFirst ? (double)b0[n] : 0.0;
        for (int k = t.k0; k < t.k1; ++k, n += pl) {
            const bool up = k + 1 < g.nz;
            double bp = 0.0, vp;
            if (MODE == kFineFirst) {
                bp = (double)b0[up ? n + pl : n];
                vp = up ? cw * bp : 0.0;
            } else {
                vp = in(up ? n + pl : n, cw);
                if (!up) vp = 0.0;
            }
            const double xw = in(n + ow, cwW), xe = in(n + oe, cwE);
            const double xs = in(n + os, cwS), xn = in(n + on, cwN);
            const double bn = MODE == kFineFirst ? bc : (double)b0[n];
            const bool fr = a.type[n] == 0;
            // a free node is never on a z face: fx = hy, fy = hx (hz = 1)
            double acc = 0.0;
            acc += ww * (vc - xw);
            acc += we * (vc - xe);
            acc += ws * (vc - xs);
            acc += wn * (vc - xn);
            acc += fz * (vc - vm);
            acc += fz * (vc - vp);
            const double v = MODE == kFineResid ? bn - acc : vc + cwo * (bn - acc);
            const mgv out = (mgv)(v * (double)fr);  // values are finite
            if (LAST) rz += bn * (double)out;
            xo[n] = out;
            vm = vc;
            vc = vp;
            bc = bp;
        }
    }
    if (LAST) {
        __shared__ double sh[kBlock / 64];
        double tsum = block_sum(rz, sh);
        if (threadIdx.x == 0) a.part_rz[blockIdx.x] = tsum;
    }
}

// ---------------------------------------------------------------------------
// Host side

static unsigned mg_grid(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    return (unsigned)(g < 1 ? 1 : g);
}

// Grid of a coarse-level kernel over nx x ny x nz nodes (see PlaneIdx).
static dim3 plane_grid(int nx, int ny, int nz) {
    return dim3((unsigned)(((int64_t)nx * ny + kBlock - 1) / kBlock), (unsigned)nz);
}
static dim3 plane_grid(const MgLevel& L) { return plane_grid(L.nx, L.ny, L.nz); }

// The coarsest operator as a dense n x n FP64 matrix (row-major) from its
// stored rows; a node without an unknown (zero row) gets a unit row and
// column, so the matrix is symmetric positive definite and its inverse keeps
// those nodes apart. act[I] = 1 for a node with an unknown.
static int coarsest_dense(const MgLevel& L, const std::vector<float>& rows, std::vector<double>& A,
                          std::vector<uint8_t>& act) {
    const int64_t n = L.n;
    act.assign(n, 0);
    for (int64_t I = 0; I < n; ++I) act[I] = rows[(size_t)I * 125 + kCenter] != 0.0f;
    A.assign((size_t)n * n, 0.0);
    for (int64_t I = 0; I < n; ++I) {
        if (!act[I]) {
            A[(size_t)I * n + I] = 1.0;
            continue;
        }
        const int i = (int)(I % L.nx), j = (int)((I / L.nx) % L.ny), k = (int)(I / ((int64_t)L.nx * L.ny));
        for (int o = 0; o < 125; ++o) {
            const float v = rows[(size_t)I * 125 + o];
            if (v == 0.0f) continue;
            const int ii = i + o % 5 - 2, jj = j + (o / 5) % 5 - 2, kk = k + o / 25 - 2;
            if (ii < 0 || ii >= L.nx || jj < 0 || jj >= L.ny || kk < 0 || kk >= L.nz) return -3;
            const int64_t K = ((int64_t)kk * L.ny + jj) * L.nx + ii;
            if (!act[K]) return -3;
            A[(size_t)I * n + K] = v;
        }
    }
    return 0;
}

// In-place Gauss-Jordan inversion of a symmetric positive definite n x n
// matrix, one pivot p per pair of launches (no pivot search: the pivots are
// the positive leading Schur complements). k_gj_save copies row p and column
// p, k_gj_step then applies
//   A[p][p] <- 1 / a,  A[p][j] <- A[p][j] / a,  A[i][p] <- -A[i][p] / a,
//   A[i][j] <- A[i][j] - A[i][p] A[p][j] / a    (a = A[p][p], i, j != p);
// after the last pivot A holds the inverse. A pivot that is not positive sets
// *bad.
__global__ __launch_bounds__(kBlock) void k_gj_save(const double* __restrict__ A, int n, int p, double* __restrict__ col,
                                                     double* __restrict__ row) {
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t >= n) return;
    col[t] = A[(size_t)t * n + p];
    row[t] = A[(size_t)p * n + t];
}

__global__ __launch_bounds__(kBlock) void k_gj_step(double* __restrict__ A, int n, int p, const double* __restrict__ col,
                                                     const double* __restrict__ row, int* __restrict__ bad) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * n) return;
    const double a = row[p];
    if (!(a > 0.0)) {
        if (e == 0) *bad = 1;
        return;
    }
    const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
    const double d = 1.0 / a;
    double v;
    if (i == p)
        v = j == p ? d : row[j] * d;
    else if (j == p)
        v = -col[i] * d;
    else
        v = A[e] - col[i] * row[j] * d;
    A[e] = v;
}

// inv = the symmetric part of the FP64 inverse in FP32, zero in the rows and
// columns of nodes without an unknown
__global__ __launch_bounds__(kBlock) void k_gj_store(const double* __restrict__ A, int n, const uint8_t* __restrict__ act,
                                                      float* __restrict__ inv) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * n) return;
    const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
    const double v = 0.5 * (A[e] + A[(size_t)j * n + i]);
    inv[e] = (act[i] && act[j]) ? (float)v : 0.0f;
}

// h->cinv = inverse of the coarsest operator L (rows: its stored rows).
static int coarsest_inverse(pic_ctx* c, const MgLevel& L, const std::vector<float>& rows, float* cinv) {
    std::vector<double> A;
    std::vector<uint8_t> act;
    if (coarsest_dense(L, rows, A, act) != 0) return -3;
    const int n = (int)L.n;
    const size_t nn = (size_t)n * n;
    // work buffer: the matrix, row and column of the pivot, the flag, the mask
    char* w = nullptr;
    const size_t off_col = nn * 8, off_row = off_col + (size_t)n * 8, off_bad = off_row + (size_t)n * 8,
                 off_act = off_bad + 256, bytes = off_act + (size_t)n;
    if (hipMalloc((void**)&w, bytes) != hipSuccess) return -2;
    double* Ad = (double*)w;
    double* col = (double*)(w + off_col);
    double* row = (double*)(w + off_row);
    int* bad = (int*)(w + off_bad);
    uint8_t* actd = (uint8_t*)(w + off_act);
    int rc = 0;
    int bad_h = 0;
    if (hipMemcpyAsync(Ad, A.data(), nn * 8, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(actd, act.data(), (size_t)n, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(bad, &bad_h, sizeof(int), hipMemcpyHostToDevice, c->stream) != hipSuccess)
        rc = -2;
    const unsigned gs = (unsigned)((n + kBlock - 1) / kBlock), ge = (unsigned)((nn + kBlock - 1) / kBlock);
    for (int p = 0; p < n && rc == 0; ++p) {
        hipLaunchKernelGGL(k_gj_save, dim3(gs), dim3(kBlock), 0, c->stream, (const double*)Ad, n, p, col, row);
        hipLaunchKernelGGL(k_gj_step, dim3(ge), dim3(kBlock), 0, c->stream, Ad, n, p, (const double*)col,
                           (const double*)row, bad);
    }
    if (rc == 0) {
        hipLaunchKernelGGL(k_gj_store, dim3(ge), dim3(kBlock), 0, c->stream, (const double*)Ad, n,
                           (const uint8_t*)actd, cinv);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            rc = -2;
        else if (bad_h)
            rc = -3;
    }
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(w);
    return rc;
}

// Classes of identical rows: ids[n] (0 for the zero row of a node without an
// unknown) and the table, kTabRow floats per class with omega / D at
// kTabInvD.
static void row_classes(const std::vector<float>& rows, int64_t n, double omega, std::vector<uint32_t>& ids,
                        std::vector<float>& tab) {
    ids.assign(n, 0);
    tab.assign(kTabRow, 0.0f);  // class 0
    std::unordered_map<uint64_t, std::vector<uint32_t>> seen;
    seen.reserve(1024);
    for (int64_t I = 0; I < n; ++I) {
        const float* r = rows.data() + (size_t)I * 125;
        if (r[kCenter] == 0.0f) continue;
        uint64_t h = 1469598103934665603ull;  // FNV-1a over the 125 coefficients
        for (int o = 0; o < 125; ++o) {
            uint32_t u;
            std::memcpy(&u, r + o, 4);
            h = (h ^ u) * 1099511628211ull;
        }
        std::vector<uint32_t>& cands = seen[h];
        uint32_t cls = 0;
        for (uint32_t c : cands)
            if (std::memcmp(tab.data() + (size_t)c * kTabRow, r, 125 * sizeof(float)) == 0) {
                cls = c;
                break;
            }
        if (cls == 0) {
            cls = (uint32_t)(tab.size() / kTabRow);
            tab.resize(tab.size() + kTabRow, 0.0f);
            float* t = tab.data() + (size_t)cls * kTabRow;
            std::memcpy(t, r, 125 * sizeof(float));
            t[kTabInvD] = (float)(omega / (double)r[kCenter]);
            double sum = 0.0;
            for (int o = 0; o < 125; ++o) sum += (double)r[o];
            t[kTabSum] = (float)sum;
            cands.push_back(cls);
        }
        ids[I] = cls;
    }
}

static void mg_release(MgHier* h) {
    if (!h) return;
    for (int l = 1; l < h->nlev; ++l) {
        if (h->lv[l].tab) (void)hipFree(h->lv[l].tab);
    }
    delete h;
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
    if (h->nlev < 2 || (int64_t)dims.back().x * dims.back().y * dims.back().z > kCoarseMax) {
        delete h;
        return -3;
    }
    h->z[0] = (mgv*)take(nn * sizeof(mgv));
    h->z[1] = (mgv*)take(nn * sizeof(mgv));
    for (int l = 0; l < h->nlev; ++l) {
        MgLevel& L = h->lv[l];
        L.nx = dims[l].x;
        L.ny = dims[l].y;
        L.nz = dims[l].z;
        L.n = (int64_t)L.nx * L.ny * L.nz;
        L.tab = nullptr;
        L.ncls = 0;
        L.zkc = 0;
        L.zblocks = 0;
        if (l >= 1 && L.nx >= 32 && L.ny >= 32)
            L.zblocks = zgrid16(L.nx, L.ny, L.nz, stencil_target(c), &L.zkc);
        if (l == 0) {
            L.id = nullptr;
            L.used = nullptr;
            L.x0 = h->z[0];
            L.x1 = h->z[1];
            L.b = nullptr;  // the finest right-hand side is passed to each V-cycle
            continue;
        }
        L.id = (uint32_t*)take(L.n * 4);
        L.used = (uint8_t*)take(L.n);
        L.x0 = (mgv*)take(L.n * sizeof(mgv));
        L.x1 = (mgv*)take(L.n * sizeof(mgv));
        L.b = (mgv*)take(L.n * sizeof(mgv));
    }
    MgLevel& Lc = h->lv[h->nlev - 1];
    h->cinv = (float*)take((size_t)Lc.n * Lc.n * 4);
    h->pre = 2;
    h->post = 2;
    h->zm_blocks = zmarch_grid(c->g.nx, c->g.ny, c->g.nz, stencil_target(c), 1, &h->zm_kc);
    // the restriction to level 1 marches in z where the coarse rows fill a
    // wavefront (an even fine width, level 1 at least 64 wide)
    h->rz_kc = 0;
    h->rz_blocks = 0;
    if (c->g.nx % 2 == 0 && h->lv[1].nx >= 64)
        h->rz_blocks = zmarch_grid(h->lv[1].nx, h->lv[1].ny, h->lv[1].nz, 1024, 1, &h->rz_kc);
    // plane grids: nz in gridDim.y, the plane size in 32-bit indices
    if (h->zm_blocks > kMaxStencilBlocks || c->g.nz > 65535 || (int64_t)c->g.nx * c->g.ny >= ((int64_t)1 << 30)) {
        delete h;
        return -3;
    }
    // Galerkin rows level by level (the largest row buffer is level 1's)
    float* rows_d = nullptr;
    if (hipMalloc((void**)&rows_d, (size_t)h->lv[1].n * 125 * sizeof(float)) != hipSuccess) {
        delete h;
        return -2;
    }
    std::vector<float> rows;
    std::vector<uint32_t> ids;
    std::vector<float> tab;
    int rc = 0;
    for (int l = 1; l < h->nlev && rc == 0; ++l) {
        MgLevel& F = h->lv[l - 1];
        MgLevel& C = h->lv[l];
        const unsigned G = mg_grid(C.n), Gg = (unsigned)((C.n + kGalBlock - 1) / kGalBlock);
        if (l == 1) {
            hipLaunchKernelGGL(k_mg_used<true>, dim3(G), dim3(kBlock), 0, c->stream, F.nx, F.ny, F.nz,
                               (const uint8_t*)c->buf.node_type, C);
            GalerkinFine src{c->g, c->buf.node_type};
            hipLaunchKernelGGL(k_mg_galerkin<GalerkinFine>, dim3(Gg), dim3(kGalBlock), 0, c->stream, src, C, rows_d);
        } else {
            hipLaunchKernelGGL(k_mg_used<false>, dim3(G), dim3(kBlock), 0, c->stream, F.nx, F.ny, F.nz,
                               (const uint8_t*)F.used, C);
            GalerkinCoarse src{F};
            hipLaunchKernelGGL(k_mg_galerkin<GalerkinCoarse>, dim3(Gg), dim3(kGalBlock), 0, c->stream, src, C,
                               rows_d);
        }
        rows.resize((size_t)C.n * 125);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(rows.data(), rows_d, rows.size() * sizeof(float), hipMemcpyDeviceToHost, c->stream) !=
                hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess) {
            rc = -2;
            break;
        }
        row_classes(rows, C.n, kOmegaC, ids, tab);
        C.ncls = (int)(tab.size() / kTabRow);
        if (hipMalloc((void**)&C.tab, tab.size() * sizeof(float)) != hipSuccess ||
            hipMemcpyAsync(C.tab, tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice, c->stream) !=
                hipSuccess ||
            hipMemcpyAsync(C.id, ids.data(), ids.size() * 4, hipMemcpyHostToDevice, c->stream) != hipSuccess) {
            rc = -2;
            break;
        }
        if (hipStreamSynchronize(c->stream) != hipSuccess) {
            rc = -2;
            break;
        }
        if (l == h->nlev - 1) rc = coarsest_inverse(c, C, rows, h->cinv);
    }
    (void)hipFree(rows_d);
    if (rc != 0) {
        mg_release(h);
        return rc;
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
    a.cg_blocks = cg_blocks;
    const int nl = h->nlev;
    const Grid& g = c->g;
    mgv* pre_out[kMgMaxLevels];  // pre-smoothed iterate per level
    mgv* res[kMgMaxLevels];      // final iterate per level
    // Jacobi sweep (resid = false) or residual (resid = true) on coarse level L
    auto sweep = [&](const MgLevel& L, bool resid, const mgv* xi, mgv* xo) {
        const float* tab = L.tab;
        if (L.zblocks) {
            if (resid)
                hipLaunchKernelGGL(k_mg_sweep_z<true>, dim3(L.zblocks), dim3(kBlock), 0, c->stream, a, L, tab, xi, xo,
                                   L.zkc);
            else
                hipLaunchKernelGGL(k_mg_sweep_z<false>, dim3(L.zblocks), dim3(kBlock), 0, c->stream, a, L, tab, xi, xo,
                                   L.zkc);
        } else if (resid) {
            hipLaunchKernelGGL(k_mg_sweep<true>, plane_grid(L), dim3(kBlock), 0, c->stream, a, L, tab, xi, xo);
        } else {
            hipLaunchKernelGGL(k_mg_sweep<false>, plane_grid(L), dim3(kBlock), 0, c->stream, a, L, tab, xi, xo);
        }
    };
    // b of level l + 1 from the residual r of level l
    // (and, on a level that is not the coarsest, its first pre-smoothing
    // sweep from zero)
    auto restrict_to = [&](int l, const mgv* r) {
        const MgLevel& F = h->lv[l];
        const MgLevel& C = h->lv[l + 1];
        const int first = l + 1 < nl - 1 ? 1 : 0;
        if (l == 0 && h->rz_blocks)
            hipLaunchKernelGGL(k_mg_restrict2z, dim3(h->rz_blocks), dim3(kBlock), 0, c->stream, a, F.nx, F.ny, F.nz,
                               r, C, first, h->rz_kc);
        else if (F.nx % 2 == 0)
            hipLaunchKernelGGL(k_mg_restrict2, plane_grid(C), dim3(kBlock), 0, c->stream, a, F.nx, F.ny, F.nz, r, C,
                               first);
        else
            hipLaunchKernelGGL(k_mg_restrict, plane_grid(C), dim3(kBlock), 0, c->stream, a, F.nx, F.ny, F.nz, r, C,
                               first);
    };
    // finest level: the convergence test and two sweeps from zero, the
    // residual, its restriction
    {
        MgLevel& L = h->lv[0];
        int t1 = timed ? tic(c, PIC_T_MG_FIRST) : -1;
        hipLaunchKernelGGL((k_mg_fine_sweep<kFineFirst, false, TB>), dim3(h->zm_blocks), dim3(kBlock), 0, c->stream, a,
                           b0, (const mgv*)nullptr, L.x0, h->zm_kc, kOmega2, kOmega1);
        toc(c, t1);
        int t2 = timed ? tic(c, PIC_T_MG_RESTRICT) : -1;
        hipLaunchKernelGGL((k_mg_fine_sweep<kFineResid, false, TB>), dim3(h->zm_blocks), dim3(kBlock), 0, c->stream, a,
                           b0, (const mgv*)L.x0, L.x1, h->zm_kc, 0.0, 0.0);
        toc(c, t2);
        restrict_to(0, (const mgv*)L.x1);
        pre_out[0] = L.x0;
    }
    // coarse levels down: pre-smoothing, residual, restriction
    for (int l = 1; l < nl - 1; ++l) {
        MgLevel& L = h->lv[l];
        mgv* cur = L.x0;  // the first sweep, written by the restriction
        mgv* oth = L.x1;
        for (int s = 1; s < h->pre; ++s) {
            sweep(L, false, cur, oth);
            mgv* t = cur;
            cur = oth;
            oth = t;
        }
        sweep(L, true, cur, oth);
        restrict_to(l, (const mgv*)oth);
        pre_out[l] = cur;
    }
    hipLaunchKernelGGL(k_mg_coarsest, dim3((unsigned)((h->lv[nl - 1].n + 3) / 4)), dim3(kBlock), 0, c->stream, a,
                       h->lv[nl - 1], (const float*)h->cinv);
    res[nl - 1] = h->lv[nl - 1].x0;
    // coarse levels up: correction, post-smoothing
    for (int l = nl - 2; l >= 1; --l) {
        MgLevel& L = h->lv[l];
        mgv* xi = pre_out[l];
        mgv* xo = xi == L.x0 ? L.x1 : L.x0;
        hipLaunchKernelGGL(k_mg_prolong<false>, plane_grid(L), dim3(kBlock), 0, c->stream, a, L.nx, L.ny, L.nz,
                           (const uint8_t*)L.used, (const mgv*)xi, xo, h->lv[l + 1], (const mgv*)res[l + 1]);
        for (int s = 0; s < h->post; ++s) {
            sweep(L, false, xo, xi);
            mgv* t = xi;
            xi = xo;
            xo = t;
        }
        res[l] = xo;
    }
    // finest level up: correction, two sweeps (the last with the r.z partials)
    MgLevel& L = h->lv[0];
    int t3 = timed ? tic(c, PIC_T_MG_CORR) : -1;
    if (g.nx % 2 == 0)
        hipLaunchKernelGGL(k_mg_prolong2, plane_grid(g.nx / 2, g.ny, g.nz), dim3(kBlock), 0, c->stream, a, g.nx, g.ny,
                           (const uint8_t*)c->buf.node_type, (const mgv*)L.x0, L.x1, h->lv[1], (const mgv*)res[1]);
    else
        hipLaunchKernelGGL(k_mg_prolong<true>, plane_grid(g.nx, g.ny, g.nz), dim3(kBlock), 0, c->stream, a, g.nx, g.ny,
                           g.nz, (const uint8_t*)c->buf.node_type, (const mgv*)L.x0, L.x1, h->lv[1], (const mgv*)res[1]);
    toc(c, t3);
    hipLaunchKernelGGL((k_mg_fine_sweep<kFinePlain, false, TB>), dim3(h->zm_blocks), dim3(kBlock), 0, c->stream, a, b0,
                       (const mgv*)L.x1, L.x0, h->zm_kc, kOmega2, 0.0);
    int t4 = timed ? tic(c, PIC_T_MG_LAST) : -1;
    hipLaunchKernelGGL((k_mg_fine_sweep<kFinePlain, true, TB>), dim3(h->zm_blocks), dim3(kBlock), 0, c->stream, a, b0,
                       (const mgv*)L.x0, L.x1, h->zm_kc, kOmega1, 0.0);
    toc(c, t4);
    *n_rz = (int)h->zm_blocks;
    return L.x1;
}

template float* mg_vcycle<double>(pic_ctx*, const double*, double*, double*, double*, int, int*, bool);
template float* mg_vcycle<float>(pic_ctx*, const float*, double*, double*, double*, int, int*, bool);

void mg_free(pic_ctx* c) {
    mg_release((MgHier*)c->mg_host);
    c->mg_host = nullptr;
}

}  // namespace pic
