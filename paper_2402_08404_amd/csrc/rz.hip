// rz.hip -- the 2D axisymmetric (r, z) 2D3V variant of the particle-mesh
// step (Sec. 2.2): node types of the axisymmetric tip, Poisson's equation in
// cylindrical finite-volume form by FP64 conjugate gradients with a
// multigrid preconditioner, the node field, gather + leapfrog push with the
// rotation back into the r-z plane, removal, the fixed-point deposit, pair
// collisions over the annular cells with Cu2+ as an ion charge state (Table
// colls, Eqs. colp, du, newv), field ionization (Eq. dfi) and
// Fowler-Nordheim emission from rings of the tip (Sec. 2.3.1). The
// discretization and the pairing are stated in pic_rz.h.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "pic_internal.hpp"
#include "pic_rz.h"

namespace pic_rz {

using pic::clampi;
using pic::Draw2;
using pic::draw2;
using pic::kBlock;
using pic::kDead;
using pic::kEps0;
using pic::kMe;
using pic::kPi;
using pic::kQe;

constexpr int kCgBlocks = 1024;  // blocks of the CG kernels (one partial each, summed in a fixed order)
constexpr uint8_t kFree = 0, kHeld0 = 1, kHeldV = 2;  // node types

constexpr uint32_t kTagPairIon = 36, kTagIon = 37;  // the (e, Cu+) class: cell shift, pair draws
constexpr int kScanBlock = 1024;  // threads of the single-block scans
constexpr int kRankSmall = 64;    // cells up to this many particles of a species: one rank per thread
constexpr int kRankLds = 4096;    // up to this many: one block sorts the cell in LDS
constexpr int kBigBlocks = 1024;  // blocks that take the larger cells in turn

struct State {
    unsigned long long absorbed[3][5];
    double rr, bb, pq, alpha, beta, rtol, rz;
    int it, maxit, done, error;
    unsigned long long n[3];       // slots in use per species
    unsigned long long next_id;    // id of the next new particle
    unsigned long long events[7];  // 1 elastic, 2 impact ionization, 3 charge exchange, 4 field ionization,
                                   // 5 double ionization of Cu, 6 ionization of Cu+
    unsigned long long injected;
    unsigned long long base_n[2], base_id;  // first electron / ion slot and first id of the stage's new particles
    unsigned long long total;      // total of the last scan
    int skip;                      // the stage's new particles did not fit
    unsigned int nbig;             // (species, cell) keys above kRankSmall particles
    unsigned long long ngrp[3];    // slots in use when the particles were grouped by cell
    unsigned long long nprod;      // entries of the product list of the collide stage
};

struct Geo {
    int nr, nz;
    double R, H;  // tip radius and height in grid units
};

__host__ __device__ inline bool inside_tip(const Geo& g, double r, double z) {
    const double zc = g.H - g.R;
    if (z < 0.0) return false;
    if (z <= zc) return r <= g.R;
    const double dz = z - zc;
    return r * r + dz * dz <= g.R * g.R;
}

// couplings of column i over pi h: radial inner, radial outer, axial
__device__ inline void couplings(int i, int nr, double& cin, double& cout, double& cax) {
    cin = i > 0 ? 2.0 * (i - 0.5) : 0.0;
    cout = i < nr - 1 ? 2.0 * (i + 0.5) : 0.0;
    const double hi = fmin(i + 0.5, nr - 1.0), lo = fmax(i - 0.5, 0.0);
    cax = hi * hi - lo * lo;
}

// (i, k) of node n = k nr + i (grids hold fewer than 2^31 nodes: 32-bit division)
__device__ inline void node_ik(int64_t n, int nr, int& i, int& k) {
    const unsigned u = (unsigned)n, d = (unsigned)nr, q = u / d;
    k = (int)q;
    i = (int)(u - q * d);
}

__global__ void k_types(Geo g, uint8_t* type) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (int64_t)g.nr * g.nz) return;
    int i, k;
    node_ik(n, g.nr, i, k);
    uint8_t t = kFree;
    if (inside_tip(g, (double)i, (double)k)) t = kHeld0;
    if (k == 0) t = kHeld0;
    if (k == g.nz - 1) t = kHeldV;
    type[n] = t;
}

// sum_j c (x_n - x_m) at a free node n (x of held neighbours as given)
__device__ inline double apply_at(const Geo& g, const double* x, int64_t n) {
    const int i = (int)((unsigned)n % (unsigned)g.nr);
    double cin, cout, cax;
    couplings(i, g.nr, cin, cout, cax);
    const double xn = x[n];
    double s = 0.0;
    if (cin != 0.0) s += cin * (xn - x[n - 1]);
    if (cout != 0.0) s += cout * (xn - x[n + 1]);
    s += cax * (xn - x[n - g.nr]);
    s += cax * (xn - x[n + g.nr]);
    return s;
}

struct CgArgs {
    Geo g;
    const uint8_t* type;
    const int64_t* rho;
    double* phi;
    double *r, *p, *q, *z;  // z: the preconditioned residual
    double* part;  // 2 * kCgBlocks partials
    State* st;
    double qscale;  // 2^-40 e / (pi eps0 h)
    double V0;
};

__device__ inline void block_reduce2(double a, double b, double* part) {
    __shared__ double sa[kBlock / 64], sb[kBlock / 64];
    a = pic::wave_sum(a);
    b = pic::wave_sum(b);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sa[w] = a;
        sb[w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0.0, tb = 0.0;
        for (int k = 0; k < kBlock / 64; ++k) {
            ta += sa[k];
            tb += sb[k];
        }
        part[2 * blockIdx.x] = ta;
        part[2 * blockIdx.x + 1] = tb;
    }
}

// sum over the blocks b of part[2 b + off] by one wavefront (four loads a
// lane issued together, then a butterfly): every lane, and every block that
// calls it, gets the same bits
__device__ inline double wave_partials(const double* part, int off) {
    static_assert(kCgBlocks % 64 == 0, "kCgBlocks must be a multiple of 64");
    const int lane = threadIdx.x & 63;
    double t[kCgBlocks / 64];
#pragma unroll
    for (int u = 0; u < kCgBlocks / 64; ++u) t[u] = part[2 * (lane + 64 * u) + off];
    double v = 0.0;
#pragma unroll
    for (int u = 0; u < kCgBlocks / 64; ++u) v += t[u];
    return pic::wave_sum(v);
}

// phi at held nodes to their values; r = b - A phi on free nodes; partials
// of r.r and of the right-hand side with the held values moved over
__global__ __launch_bounds__(kBlock) void k_cg_init(CgArgs a) {
    const int64_t nn = (int64_t)a.g.nr * a.g.nz;
    double rr = 0.0, bb = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += (int64_t)gridDim.x * blockDim.x) {
        const uint8_t t = a.type[n];
        if (t != kFree) {
            a.phi[n] = t == kHeldV ? a.V0 : 0.0;
            a.r[n] = 0.0;
            a.p[n] = 0.0;
        }
    }
    // the held values written above may not be visible yet to other blocks,
    // so a held neighbour's value is formed from its type
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += (int64_t)gridDim.x * blockDim.x) {
        if (a.type[n] != kFree) continue;
        const int i = (int)((unsigned)n % (unsigned)a.g.nr);
        double cin, cout, cax;
        couplings(i, a.g.nr, cin, cout, cax);
        const double b = (double)a.rho[n] * a.qscale;
        const int64_t nb[4] = {n - 1, n + 1, n - a.g.nr, n + a.g.nr};
        const double cb[4] = {cin, cout, cax, cax};
        const double xn = a.phi[n];
        double ax = 0.0, lift = 0.0;
        for (int k = 0; k < 4; ++k) {
            if (cb[k] == 0.0) continue;
            const int64_t m = nb[k];
            const uint8_t tm = a.type[m];
            const double xm = tm == kFree ? a.phi[m] : (tm == kHeldV ? a.V0 : 0.0);
            ax += cb[k] * (xn - xm);
            if (tm != kFree) lift += cb[k] * xm;
        }
        const double r = b - ax;
        a.r[n] = r;
        rr += r * r;
        const double be = b + lift;
        bb += be * be;
    }
    block_reduce2(rr, bb, a.part);
}

// (one wavefront) rr, bb from the partials
__global__ void k_cg_start(CgArgs a, double rtol, int maxit) {
    const double rr = wave_partials(a.part, 0), bb = wave_partials(a.part, 1);
    if (threadIdx.x == 0) {
        State* st = a.st;
        st->rr = rr;
        st->bb = bb;
        st->rtol = rtol;
        st->maxit = maxit;
        st->it = 0;
        st->done = (rr <= rtol * rtol * bb || bb == 0.0) ? 1 : 0;
    }
}

// q = A p; partial p.q
__global__ __launch_bounds__(kBlock) void k_cg_ap(CgArgs a) {
    if (a.st->done) return;
    const int64_t nn = (int64_t)a.g.nr * a.g.nz;
    double pq = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += (int64_t)gridDim.x * blockDim.x) {
        if (a.type[n] != kFree) continue;
        const double q = apply_at(a.g, a.p, n);
        a.q[n] = q;
        pq += a.p[n] * q;
    }
    block_reduce2(pq, 0.0, a.part);
}

// phi += alpha p, r -= alpha q (alpha from the partials, every block the same
// sum in the same order); partial r.r
__global__ __launch_bounds__(kBlock) void k_cg_update(CgArgs a) {
    if (a.st->done) return;
    __shared__ double alpha;
    if (threadIdx.x < 64) {
        const double pq = wave_partials(a.part, 0);
        if (threadIdx.x == 0) alpha = a.st->rz / pq;
    }
    __syncthreads();
    const int64_t nn = (int64_t)a.g.nr * a.g.nz;
    double rr = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += (int64_t)gridDim.x * blockDim.x) {
        if (a.type[n] != kFree) continue;
        a.phi[n] += alpha * a.p[n];
        const double r = a.r[n] - alpha * a.q[n];
        a.r[n] = r;
        rr += r * r;
    }
    block_reduce2(rr, 0.0, a.part + 2 * kCgBlocks);
}

// (one wavefront) r.r from the partials, convergence
__global__ void k_cg_check(CgArgs a) {
    State* st = a.st;
    if (st->done) return;
    const double rr = wave_partials(a.part + 2 * kCgBlocks, 0);
    if (threadIdx.x != 0) return;
    st->rr = rr;
    st->it += 1;
    if (rr <= st->rtol * st->rtol * st->bb || st->it >= st->maxit) st->done = 1;
}

// partials of r.z; with first set, also p = z
__global__ __launch_bounds__(kBlock) void k_pcg_rz(CgArgs a, int first) {
    if (a.st->done) return;
    const int64_t nn = (int64_t)a.g.nr * a.g.nz;
    double rz = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += (int64_t)gridDim.x * blockDim.x) {
        if (a.type[n] != kFree) continue;
        const double z = a.z[n];
        rz += a.r[n] * z;
        if (first) a.p[n] = z;
    }
    block_reduce2(rz, 0.0, a.part);
}

// (one wavefront) beta = r.z / previous r.z (first: only r.z)
__global__ void k_pcg_beta(CgArgs a, int first) {
    State* st = a.st;
    if (st->done) return;
    const double rz = wave_partials(a.part, 0);
    if (threadIdx.x != 0) return;
    st->beta = first ? 0.0 : rz / st->rz;
    st->rz = rz;
}

__global__ __launch_bounds__(kBlock) void k_cg_p(CgArgs a) {
    if (a.st->done) return;
    const double beta = a.st->beta;
    const int64_t nn = (int64_t)a.g.nr * a.g.nz;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += (int64_t)gridDim.x * blockDim.x)
        if (a.type[n] == kFree) a.p[n] = a.z[n] + beta * a.p[n];
}

// ---------------------------------------------------------------------------
// Multigrid preconditioner of the CG: one V-cycle z = M r of the error
// equation (held nodes at zero). Level l has nr_l x nz_l nodes; a dimension
// is halved (node I of the coarse level at node 2 I of the finer) while its
// cell count is even and at least 4, until a level has at most kMgDirectMax
// nodes; the coarse operator is the same finite
// volume discretization at the coarse spacings H_r = 2^a h, H_z = 2^b h,
// in units of pi eps0 h: radial couplings 2^b 2 (I -+ 1/2), axial couplings
// 2^(2a-b) (r_hi^2 - r_lo^2) in coarse index units. A coarse node is held if
// the finer node at its place is. Prolongation is bilinear, restriction its
// transpose (the residual is an integrated charge, so it is summed). Damped
// Jacobi (omega = 4/5) smooths, two sweeps before and two after; the coarsest
// level is solved exactly when it has at most kMgDirectMax nodes (its inverse
// from the set-up), else (a level that cannot be halved further) swept
// kMgCoarseSweeps times from zero in LDS when it has at most kMgCoarseMax
// nodes, else smoothed like the others. The cycle is a fixed symmetric linear
// operator, as CG needs.
constexpr int kMgMaxLevels = 16;
constexpr int kMgCoarseMax = 2048;
constexpr int kMgCoarseSweeps = 64;
constexpr int kMgDirectMax = 64;  // the coarsening stops at this many nodes; such a level is solved exactly
constexpr double kMgOmega = 0.8;

struct Lv {
    int nr, nz;
    double fr, fa;        // coupling factors 2^b, 2^(2a - b)
    const uint8_t* type;  // 0 free
};

// sum_j c (x_n - x_m) over the neighbours (held ones at zero) and the
// diagonal, at node n = (i, k); xv(m, i, k) gives the value of node m = (i, k)
// (the neighbours' types and values are read unconditionally, at indices
// clamped into the grid, so that the loads are in flight together)
template <class X>
__device__ inline double lv_apply_f(const Lv& L, int64_t n, int i, int k, double& diag, X xv) {
    const double cin = i > 0 ? L.fr * 2.0 * (i - 0.5) : 0.0;
    const double cout = i < L.nr - 1 ? L.fr * 2.0 * (i + 0.5) : 0.0;
    const double hi = fmin(i + 0.5, L.nr - 1.0), lo = fmax(i - 0.5, 0.0);
    const double cax = L.fa * (hi * hi - lo * lo);
    const bool iw = i > 0, ie = i < L.nr - 1, is = k > 0, in = k < L.nz - 1;
    const int64_t mw = iw ? n - 1 : n, me = ie ? n + 1 : n, ms = is ? n - L.nr : n, mn = in ? n + L.nr : n;
    const uint8_t tw = L.type[mw], te = L.type[me], ts = L.type[ms], tn = L.type[mn];
    const double xn = xv(n, i, k);
    const double xw = xv(mw, iw ? i - 1 : i, k), xe = xv(me, ie ? i + 1 : i, k);
    const double xs = xv(ms, i, is ? k - 1 : k), xq = xv(mn, i, in ? k + 1 : k);
    double s = 0.0;
    if ((cin != 0.0) & (tw == kFree)) s -= cin * xw;
    if ((cout != 0.0) & (te == kFree)) s -= cout * xe;
    if (is & (ts == kFree)) s -= cax * xs;
    if (in & (tn == kFree)) s -= cax * xq;
    diag = cin + cout + 2.0 * cax;
    return s + diag * xn;
}

__device__ inline double lv_apply(const Lv& L, const double* x, int64_t n, int i, int k, double& diag) {
    return lv_apply_f(L, n, i, k, diag, [&](int64_t m, int, int) { return x[m]; });
}

__device__ inline double lv_apply(const Lv& L, const double* x, int64_t n, double& diag) {
    int i, k;
    node_ik(n, L.nr, i, k);
    return lv_apply(L, x, n, i, k, diag);
}

// the diagonal of a node of column i
__device__ inline double lv_diag(const Lv& L, int i) {
    const double cin = i > 0 ? L.fr * 2.0 * (i - 0.5) : 0.0;
    const double cout = i < L.nr - 1 ? L.fr * 2.0 * (i + 0.5) : 0.0;
    const double hi = fmin(i + 0.5, L.nr - 1.0), lo = fmax(i - 0.5, 0.0);
    const double cax = L.fa * (hi * hi - lo * lo);
    return cin + cout + 2.0 * cax;
}

// The level operations over nodes n0, n0 + stride, ... (a grid-stride loop
// in the kernels of one level, a block-stride loop in k_mg_lds).

// y = x + omega D^-1 (b - A x) at free nodes (zero_x: x taken as zero)
__device__ inline void mg_jacobi(const Lv& L, const double* x, double* y, const double* b, int zero_x, int64_t n0,
                                 int64_t stride) {
    const int64_t nn = (int64_t)L.nr * L.nz;
    for (int64_t n = n0; n < nn; n += stride) {
        if (L.type[n] != kFree) continue;
        double d;
        if (zero_x) {
            lv_apply(L, b, n, d);  // the diagonal only
            y[n] = kMgOmega * b[n] / d;
        } else {
            const double ax = lv_apply(L, x, n, d);
            y[n] = x[n] + kMgOmega * (b[n] - ax) / d;
        }
    }
}

__device__ inline void mg_resid(const Lv& L, const double* x, const double* b, double* t, int64_t n0,
                                int64_t stride) {
    const int64_t nn = (int64_t)L.nr * L.nz;
    for (int64_t n = n0; n < nn; n += stride) {
        if (L.type[n] != kFree) continue;
        double d;
        t[n] = b[n] - lv_apply(L, x, n, d);
    }
}

__global__ __launch_bounds__(kBlock) void k_mg_jacobi(Lv L, const double* x, double* y, const double* b, int zero_x,
                                                       const State* st) {
    if (st->done) return;
    mg_jacobi(L, x, y, b, zero_x, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
}

// b_c = R t (sr, sz: 2 where the dimension is halved, else 1)
__device__ inline void mg_restrict(const Lv& F, const Lv& Cl, const double* t, double* bc, int sr, int sz,
                                   int64_t n0, int64_t stride) {
    const int64_t nn = (int64_t)Cl.nr * Cl.nz;
    for (int64_t n = n0; n < nn; n += stride) {
        if (Cl.type[n] != kFree) continue;
        int I, K;
        node_ik(n, Cl.nr, I, K);
        const int i0 = sr * I, k0 = sz * K;
        double s = 0.0;
        for (int dk = -(sz - 1); dk <= sz - 1; ++dk) {
            const int k = k0 + dk;
            if (k < 0 || k >= F.nz) continue;
            const double wk = dk == 0 ? 1.0 : 0.5;
            for (int di = -(sr - 1); di <= sr - 1; ++di) {
                const int i = i0 + di;
                if (i < 0 || i >= F.nr) continue;
                const double wi = di == 0 ? 1.0 : 0.5;
                const int64_t m = (int64_t)k * F.nr + i;
                if (F.type[m] == kFree) s += wi * wk * t[m];
            }
        }
        bc[n] = s;
    }
}

// x_f += P x_c at free fine nodes
__device__ inline void mg_prolong(const Lv& F, const Lv& Cl, const double* xc, double* xf, int sr, int sz,
                                  int64_t n0, int64_t stride) {
    const int64_t nn = (int64_t)F.nr * F.nz;
    for (int64_t n = n0; n < nn; n += stride) {
        if (F.type[n] != kFree) continue;
        int i, k;
        node_ik(n, F.nr, i, k);
        int I0 = i, I1 = i, K0 = k, K1 = k;
        if (sr == 2) {
            I0 = i >> 1;
            I1 = (i + 1) >> 1;
        }
        if (sz == 2) {
            K0 = k >> 1;
            K1 = (k + 1) >> 1;
        }
        const double wi = I0 == I1 ? 1.0 : 0.5, wk = K0 == K1 ? 1.0 : 0.5;
        auto at = [&](int I, int K) {
            const int64_t m = (int64_t)K * Cl.nr + I;
            return Cl.type[m] == kFree ? xc[m] : 0.0;
        };
        double v = at(I0, K0);
        if (I1 != I0) v += at(I1, K0);
        if (K1 != K0) {
            v += at(I0, K1);
            if (I1 != I0) v += at(I1, K1);
        }
        xf[n] += wi * wk * v;
    }
}

// Fused level kernels of the large levels (one launch instead of two or
// three; the values of every node are those of the separate passes).

// y = two sweeps from zero: the first sweep's value omega b_m / d_m is formed
// at the node and its neighbours
__global__ __launch_bounds__(kBlock) void k_mg_smooth2(Lv L, const double* b, double* y, const State* st) {
    if (st->done) return;
    const int64_t nn = (int64_t)L.nr * L.nz;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += (int64_t)gridDim.x * blockDim.x) {
        if (L.type[n] != kFree) continue;
        int i, k;
        node_ik(n, L.nr, i, k);
        double d;
        const double ax =
            lv_apply_f(L, n, i, k, d, [&](int64_t m, int im, int) { return kMgOmega * b[m] / lv_diag(L, im); });
        const double x1 = kMgOmega * b[n] / d;
        y[n] = x1 + kMgOmega * (b[n] - ax) / d;
    }
}

// The fused kernels read every value a node needs up front (indices clamped
// into the grid, the ones outside it marked not free), so the loads are in
// flight together; the arithmetic, in the same order, is that of lv_apply,
// mg_restrict and mg_prolong. SR, SZ: 2 where the dimension is halved.

// the stencil of lv_apply at column i from a patch: f[c], x[c] the node,
// f/x[w], [e] its radial and [s], [nn] its axial neighbours (f: free)
__device__ inline double patch_apply(const Lv& L, int i, const bool* f, const double* x, int c, int w, int e, int s,
                                     int nn, double& diag) {
    const double cin = i > 0 ? L.fr * 2.0 * (i - 0.5) : 0.0;
    const double cout = i < L.nr - 1 ? L.fr * 2.0 * (i + 0.5) : 0.0;
    const double hi = fmin(i + 0.5, L.nr - 1.0), lo = fmax(i - 0.5, 0.0);
    const double cax = L.fa * (hi * hi - lo * lo);
    double a = 0.0;
    if (cin != 0.0 && f[w]) a -= cin * x[w];
    if (cout != 0.0 && f[e]) a -= cout * x[e];
    if (f[s]) a -= cax * x[s];
    if (f[nn]) a -= cax * x[nn];
    diag = cin + cout + 2.0 * cax;
    return a + diag * x[c];
}

// b_c = R (b - A x): the residual formed at each fine node the restriction
// reads, from the patch of fine nodes within one node of them
template <int SR, int SZ>
__global__ __launch_bounds__(kBlock) void k_mg_resid_restrict(Lv F, Lv Cl, const double* x, const double* b,
                                                               double* bc, const State* st) {
    if (st->done) return;
    constexpr int RI = SR - 1, RK = SZ - 1, PW = 2 * RI + 3, PH = 2 * RK + 3;
    const int64_t nn = (int64_t)Cl.nr * Cl.nz;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += (int64_t)gridDim.x * blockDim.x) {
        if (Cl.type[n] != kFree) continue;
        int I, K;
        node_ik(n, Cl.nr, I, K);
        const int i0 = SR * I, k0 = SZ * K;
        bool f[PH * PW];
        double xp[PH * PW], bp[PH * PW];
#pragma unroll
        for (int pk = 0; pk < PH; ++pk)
#pragma unroll
            for (int pi = 0; pi < PW; ++pi) {
                const int i = i0 + pi - RI - 1, k = k0 + pk - RK - 1;
                const bool in = i >= 0 && i < F.nr && k >= 0 && k < F.nz;
                const int64_t m = in ? (int64_t)k * F.nr + i : 0;
                const uint8_t t = F.type[m];  // loaded whether or not inside: no branch between the loads
                f[pk * PW + pi] = in & (t == kFree);
                xp[pk * PW + pi] = x[m];
                const bool inner = pi >= 1 && pi <= PW - 2 && pk >= 1 && pk <= PH - 2;
                bp[pk * PW + pi] = inner ? b[m] : 0.0;
            }
        double s = 0.0;
#pragma unroll
        for (int dk = -RK; dk <= RK; ++dk) {
            const double wk = dk == 0 ? 1.0 : 0.5;
#pragma unroll
            for (int di = -RI; di <= RI; ++di) {
                const double wi = di == 0 ? 1.0 : 0.5;
                const int c = (dk + RK + 1) * PW + di + RI + 1;
                if (!f[c]) continue;
                double d;
                const double ax = patch_apply(F, i0 + di, f, xp, c, c - 1, c + 1, c - PW, c + PW, d);
                const double t = bp[c] - ax;
                s += wi * wk * t;
            }
        }
        bc[n] = s;
    }
}

// the bilinear correction P x_c at fine node (i, k) (free); SR, SZ as above
template <int SR, int SZ>
__device__ inline double mg_corr(const Lv& Cl, const double* xc, int i, int k) {
    const int I0 = SR == 2 ? i >> 1 : i, I1 = SR == 2 ? (i + 1) >> 1 : i;
    const int K0 = SZ == 2 ? k >> 1 : k, K1 = SZ == 2 ? (k + 1) >> 1 : k;
    const double wi = I0 == I1 ? 1.0 : 0.5, wk = K0 == K1 ? 1.0 : 0.5;
    const int64_t m00 = (int64_t)K0 * Cl.nr + I0, m10 = (int64_t)K0 * Cl.nr + I1;
    const int64_t m01 = (int64_t)K1 * Cl.nr + I0, m11 = (int64_t)K1 * Cl.nr + I1;
    const double a00 = Cl.type[m00] == kFree ? xc[m00] : 0.0;
    const double a10 = Cl.type[m10] == kFree ? xc[m10] : 0.0;
    const double a01 = Cl.type[m01] == kFree ? xc[m01] : 0.0;
    const double a11 = Cl.type[m11] == kFree ? xc[m11] : 0.0;
    double v = a00;
    if (I1 != I0) v += a10;
    if (K1 != K0) {
        v += a01;
        if (I1 != I0) v += a11;
    }
    return wi * wk * v;
}

// y = one sweep from x + P x_c (the corrected value formed at the node and
// its neighbours; x itself is not written)
template <int SR, int SZ>
__global__ __launch_bounds__(kBlock) void k_mg_prolong_smooth(Lv F, Lv Cl, const double* xc, const double* x,
                                                               double* y, const double* b, const State* st) {
    if (st->done) return;
    const int64_t nn = (int64_t)F.nr * F.nz;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += (int64_t)gridDim.x * blockDim.x) {
        if (F.type[n] != kFree) continue;
        int i, k;
        node_ik(n, F.nr, i, k);
        // the node (0) and its neighbours west, east, south, north (1-4), clamped into the grid
        const int di[5] = {0, -1, 1, 0, 0}, dk[5] = {0, 0, 0, -1, 1};
        bool f[5];
        double v[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const int iq = i + di[q], kq = k + dk[q];
            const bool in = iq >= 0 && iq < F.nr && kq >= 0 && kq < F.nz;
            const int ic = in ? iq : i, kc = in ? kq : k;
            const int64_t m = (int64_t)kc * F.nr + ic;
            const uint8_t t = F.type[m];
            f[q] = in & (t == kFree);
            v[q] = x[m] + mg_corr<SR, SZ>(Cl, xc, ic, kc);
        }
        double d;
        const double ax = patch_apply(F, i, f, v, 0, 1, 2, 3, 4, d);
        y[n] = v[0] + kMgOmega * (b[n] - ax) / d;
    }
}

// x = A_c^-1 b on the coarsest level from its inverse (nc x nc, zero rows and
// columns at held nodes), at free nodes; the sum in column order
__device__ inline void mg_direct(const Lv& C, const double* inv, const double* b, double* x, int64_t n0,
                                 int64_t stride) {
    const int nc = C.nr * C.nz;
    for (int64_t j = n0; j < nc; j += stride) {
        if (C.type[j] != kFree) continue;
        double s = 0.0;
        for (int k = 0; k < nc; ++k) {
            const double w = inv[j * nc + k], bk = b[k];  // read unconditionally (b of held nodes is never used)
            if (C.type[k] == kFree) s += w * bk;
        }
        x[j] = s;
    }
}

// the coarsest level: kMgCoarseSweeps Jacobi sweeps from zero, in LDS, one block
__device__ inline void mg_coarse(const Lv& L, const double* b, double* x, double (*xs)[kMgCoarseMax]) {
    const int nn = L.nr * L.nz;
    for (int n = threadIdx.x; n < nn; n += blockDim.x) xs[0][n] = 0.0;
    __syncthreads();
    int cur = 0;
    for (int sweep = 0; sweep < kMgCoarseSweeps; ++sweep) {
        for (int n = threadIdx.x; n < nn; n += blockDim.x) {
            if (L.type[n] != kFree) {
                xs[cur ^ 1][n] = 0.0;
                continue;
            }
            double d;
            const double ax = lv_apply(L, xs[cur], n, d);
            xs[cur ^ 1][n] = xs[cur][n] + kMgOmega * (b[n] - ax) / d;
        }
        __syncthreads();
        cur ^= 1;
    }
    for (int n = threadIdx.x; n < nn; n += blockDim.x) x[n] = xs[cur][n];
}

__global__ __launch_bounds__(kBlock) void k_mg_coarse(Lv L, const double* b, double* x, const double* inv,
                                                       const State* st) {
    if (st->done) return;
    __shared__ double xs[2][kMgCoarseMax];
    if (inv) mg_direct(L, inv, b, x, threadIdx.x, blockDim.x);
    else mg_coarse(L, b, x, xs);
}

// The levels from l0 down in one block with every vector in LDS, when their
// nodes add up to at most kMgLdsNodes (separate launches per level cost more
// than the whole work of these levels): the right-hand side of level l0 is
// read once, its x_b written once at the end, and each phase is one pass of
// the block over a level's nodes between barriers. The arithmetic of every
// node is that of the level kernels; the residual of a level is kept in its
// x_a, free after the pre-smoothing.
constexpr int kMgLdsNodes = 2560;
constexpr int kMgLdsBlock = 1024;

struct MgLds {
    int l0, levels;
    Lv lv[kMgMaxLevels];  // node types in global memory
    int off[kMgMaxLevels], sr[kMgMaxLevels], sz[kMgMaxLevels];
    const double* b;    // level l0
    double* x;          // level l0 (x_b), written at free nodes
    const double* inv;  // inverse of the coarsest operator, or null (sweeps)
};

__global__ __launch_bounds__(kMgLdsBlock) void k_mg_lds(MgLds m, const State* st) {
    if (st->done) return;
    __shared__ double sb[kMgLdsNodes], sxa[kMgLdsNodes], sxb[kMgLdsNodes];
    __shared__ double sinv[kMgDirectMax * kMgDirectMax];
    __shared__ uint8_t sty[kMgLdsNodes];
    const int64_t t0 = threadIdx.x, T = blockDim.x;
    const int last = m.levels - 1;
    auto lv = [&](int l) {
        Lv L = m.lv[l];
        L.type = sty + m.off[l];
        return L;
    };
    // the staging loops are unrolled so that several loads are in flight
    // before the first LDS write (one loop over the types of all levels)
    {
        const int ntot = m.off[last] + m.lv[last].nr * m.lv[last].nz;
#pragma unroll 4
        for (int q = (int)t0; q < ntot; q += (int)T) {
            int l = m.l0;
            while (l < last && q >= m.off[l + 1]) ++l;
            sty[q] = m.lv[l].type[q - m.off[l]];
        }
        const int nb = m.lv[m.l0].nr * m.lv[m.l0].nz;
#pragma unroll 4
        for (int q = (int)t0; q < nb; q += (int)T) {
            const double v = m.b[q];
            const uint8_t t = m.lv[m.l0].type[q];
            sb[q] = t == kFree ? v : 0.0;
        }
        if (m.inv) {
            const int nc = m.lv[last].nr * m.lv[last].nz;
#pragma unroll 4
            for (int q = (int)t0; q < nc * nc; q += (int)T) sinv[q] = m.inv[q];
        }
    }
    __syncthreads();
    for (int l = m.l0; l < last; ++l) {
        const Lv F = lv(l), Cl = lv(l + 1);
        double *b = sb + m.off[l], *xa = sxa + m.off[l], *xb = sxb + m.off[l];
        mg_jacobi(F, xb, xa, b, 1, t0, T);
        __syncthreads();
        mg_jacobi(F, xa, xb, b, 0, t0, T);
        __syncthreads();
        mg_resid(F, xb, b, xa, t0, T);
        __syncthreads();
        mg_restrict(F, Cl, xa, sb + m.off[l + 1], m.sr[l], m.sz[l], t0, T);
        __syncthreads();
    }
    {
        const Lv C = lv(last);
        double *b = sb + m.off[last], *xa = sxa + m.off[last], *xb = sxb + m.off[last];
        if (m.inv) {
            mg_direct(C, sinv, b, xb, t0, T);
            __syncthreads();
        } else {
            const int sweeps = (int64_t)C.nr * C.nz <= kMgCoarseMax ? kMgCoarseSweeps : 4;  // even: the result in x_b
            for (int k = 0; k < sweeps; k += 2) {
                mg_jacobi(C, xb, xa, b, k == 0, t0, T);
                __syncthreads();
                mg_jacobi(C, xa, xb, b, 0, t0, T);
                __syncthreads();
            }
        }
    }
    for (int l = last - 1; l >= m.l0; --l) {
        const Lv F = lv(l), Cl = lv(l + 1);
        double *b = sb + m.off[l], *xa = sxa + m.off[l], *xb = sxb + m.off[l];
        mg_prolong(F, Cl, sxb + m.off[l + 1], xb, m.sr[l], m.sz[l], t0, T);
        __syncthreads();
        mg_jacobi(F, xb, xa, b, 0, t0, T);
        __syncthreads();
        mg_jacobi(F, xa, xb, b, 0, t0, T);
        __syncthreads();
    }
    const int64_t nn = (int64_t)m.lv[m.l0].nr * m.lv[m.l0].nz;
    for (int64_t n = t0; n < nn; n += T)
        if (sty[n] == kFree) m.x[n] = sxb[n];
}

// The guess of a step solve from the two previous step potentials: phi
// (the last) becomes 2 phi - prev at free nodes and prev takes the last
// (two = 0: only prev takes it, the first step)
__global__ void k_extrap(const uint8_t* type, double* phi, double* prev, int64_t nn, int two) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn || type[n] != kFree) return;
    const double t = phi[n];
    if (two) phi[n] = 2.0 * t - prev[n];
    prev[n] = t;
}

__global__ void k_field(Geo g, const double* phi, double h, double* E) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (int64_t)g.nr * g.nz) return;
    int i, k;
    node_ik(n, g.nr, i, k);
    double er = 0.0, ez;
    if (i > 0 && i < g.nr - 1) er = -(phi[n + 1] - phi[n - 1]) / (2.0 * h);
    if (k == 0) ez = -(phi[n + g.nr] - phi[n]) / h;
    else if (k == g.nz - 1) ez = -(phi[n] - phi[n - g.nr]) / h;
    else ez = -(phi[n + g.nr] - phi[n - g.nr]) / (2.0 * h);
    E[2 * n] = er;
    E[2 * n + 1] = ez;
}

struct PushArgs {
    Geo g;
    double *r, *z, *vr, *vt, *vz;
    uint32_t* id;
    const uint8_t* charge;  // ions with Cu2+: charge states (the kick scales with them)
    const double* E;
    double kq;  // (q / m) dt^2 / h
    int sp;
    State* st;
};

__global__ __launch_bounds__(kBlock) void k_push(PushArgs a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)a.st->n[a.sp]) return;
    // the state is read with the id (not after it), so the loads are in flight together
    const uint32_t id = a.id[p];
    double r = a.r[p], z = a.z[p], vr = a.vr[p], vt = a.vt[p], vz = a.vz[p];
    const double qs = a.charge ? (double)a.charge[p] : 1.0;
    if (id == kDead) return;
    const Geo& g = a.g;
    const double kq = a.charge ? a.kq * qs : a.kq;
    if (kq != 0.0) {
        const int i = clampi((int)floor(r), 0, g.nr - 2), k = clampi((int)floor(z), 0, g.nz - 2);
        const double fr = r - i, fz = z - k;
        const int64_t n0 = (int64_t)k * g.nr + i;
        const double w00 = (1 - fr) * (1 - fz), w10 = fr * (1 - fz), w01 = (1 - fr) * fz, w11 = fr * fz;
        const double er = w00 * a.E[2 * n0] + w10 * a.E[2 * (n0 + 1)] + w01 * a.E[2 * (n0 + g.nr)] +
                          w11 * a.E[2 * (n0 + g.nr + 1)];
        const double ez = w00 * a.E[2 * n0 + 1] + w10 * a.E[2 * (n0 + 1) + 1] + w01 * a.E[2 * (n0 + g.nr) + 1] +
                          w11 * a.E[2 * (n0 + g.nr + 1) + 1];
        vr += kq * er;
        vz += kq * ez;
    }
    const double x = r + vr, y = vt;
    z += vz;
    const double rn = sqrt(x * x + y * y);
    double c = 1.0, s = 0.0;
    if (rn > 0.0) {
        c = x / rn;
        s = y / rn;
    }
    const double vrn = c * vr + s * vt, vtn = -s * vr + c * vt;
    a.r[p] = rn;
    a.z[p] = z;
    a.vr[p] = vrn;
    a.vt[p] = vtn;
    a.vz[p] = vz;
    int code = 0;
    if (z <= 0.0) code = 1;
    else if (z >= (double)(g.nz - 1)) code = 2;
    else if (rn >= (double)(g.nr - 1)) code = 3;
    else if (inside_tip(g, rn, z)) code = 4;
    if (code) {
        a.id[p] = kDead;
        atomicAdd(&a.st->absorbed[a.sp][code], 1ull);
    }
}

__global__ void k_scale_copy(double* y, const double* x, double a, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i];
}

__global__ void k_zero_rho(int64_t* rho, int64_t nn) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n < nn) rho[n] = 0;
}

// tail: the slots from st->ngrp[sp] on (those added after the grouping)
__global__ __launch_bounds__(kBlock) void k_deposit(Geo g, const double* r, const double* z, const uint32_t* id,
                                                     const State* st, int sp, int64_t sign0, int64_t* rho, int tail,
                                                     const uint8_t* charge) {
    const int64_t p = (tail ? (int64_t)st->ngrp[sp] : 0) + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)st->n[sp]) return;
    const uint32_t pid = id[p];
    const double R = r[p], Z = z[p];
    const int64_t sign = charge ? sign0 * (int64_t)charge[p] : sign0;
    if (pid == kDead) return;
    const int i = clampi((int)floor(R), 0, g.nr - 2), k = clampi((int)floor(Z), 0, g.nz - 2);
    const int64_t qr = pic::quantize(R - i, 20), qz = pic::quantize(Z - k, 20);
    const int64_t one = 1 << 20;
    const int64_t n0 = (int64_t)k * g.nr + i;
    unsigned long long* q = (unsigned long long*)rho;
    atomicAdd(q + n0, (unsigned long long)(sign * (one - qr) * (one - qz)));
    atomicAdd(q + n0 + 1, (unsigned long long)(sign * qr * (one - qz)));
    atomicAdd(q + n0 + g.nr, (unsigned long long)(sign * (one - qr) * qz));
    atomicAdd(q + n0 + g.nr + 1, (unsigned long long)(sign * qr * qz));
}

// alive particles (with q, those of charge state 2): per-thread counts over
// a grid-stride loop, one atomic per block
__global__ __launch_bounds__(kBlock) void k_counts(const uint32_t* id, const State* st, int sp,
                                                    unsigned long long* out, const uint8_t* q = nullptr) {
    __shared__ unsigned long long sh[kBlock / 64];
    const int64_t n = (int64_t)st->n[sp];
    unsigned long long cnt = 0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
        cnt += (id[p] != kDead && (!q || q[p] == 2)) ? 1ull : 0ull;
    cnt = pic::wave_sum(cnt);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int q = 0; q < kBlock / 64; ++q) t += sh[q];
        if (t) atomicAdd(out, t);
    }
}

__global__ void k_qsum(const int64_t* rho, int64_t nn, unsigned long long* out) {
    long long s = 0;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += (int64_t)gridDim.x * blockDim.x)
        s += rho[n];
    s = pic::wave_sum(s);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(out, (unsigned long long)s);
}

// ---------------------------------------------------------------------------
// Initial ids: none free; next_id one above the largest.
__global__ __launch_bounds__(kBlock) void k_check_ids(const uint32_t* id, int64_t n, State* st) {
    __shared__ unsigned long long wm[kBlock / 64];
    // grid-stride: the largest id + 1 with one atomic per block
    unsigned long long m = 0;
    int bad = 0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t v = id[p];
        if (v == kDead) bad = 1;
        else m = (unsigned long long)v + 1ull > m ? (unsigned long long)v + 1ull : m;
    }
    if (bad) atomicOr(&st->skip, 1);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(m, o, 64);
        m = y > m ? y : m;
    }
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) m = wm[w] > m ? wm[w] : m;
        m = wm[0] > m ? wm[0] : m;
        if (m) atomicMax(&st->next_id, m);
    }
}

// Initial ion charge states: 1 or 2.
__global__ void k_check_charge(const uint8_t* q, int64_t n, State* st) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n && q[p] != 1 && q[p] != 2) atomicOr(&st->skip, 1);
}

// Exclusive prefix sums of m counts in one block of kScanBlock threads, in
// chunks of 4 kScanBlock (each thread a run of four, wavefront shuffles, the
// wavefront totals in shared memory); the grand total goes to st->total.
template <typename TO>
__global__ __launch_bounds__(kScanBlock) void k_scan(const uint32_t* in, TO* out, int64_t m, State* st,
                                                     const unsigned long long* mdev = nullptr, int per = 1) {
    // mdev: the length is ceil(*mdev / per), at most m (a list whose length
    // only the device knows)
    if (mdev) m = std::min<int64_t>(m, (int64_t)((*mdev + per - 1) / per));
    __shared__ unsigned long long wsum[kScanBlock / 64];
    __shared__ unsigned long long carry_s;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int64_t base = 0; base < m; base += 4 * kScanBlock) {
        const int64_t i0 = base + 4 * (int64_t)threadIdx.x;
        unsigned long long v[4], run = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = i0 + k < m ? (unsigned long long)in[i0 + k] : 0ull;
            run += v[k];
        }
        unsigned long long x = run;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned long long y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        unsigned long long pre = carry_s, tot = 0;
        for (int q = 0; q < kScanBlock / 64; ++q) {
            pre += q < w ? wsum[q] : 0ull;
            tot += wsum[q];
        }
        pre += x - run;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (i0 + k < m) out[i0 + k] = (TO)pre;
            pre += v[k];
        }
        __syncthreads();
        if (threadIdx.x == 0) carry_s += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) st->total = carry_s;
}

// The same over many blocks: k_scan_sums leaves the sum of every chunk of
// kScanChunk counts, k_scan (one block) their exclusive prefix and the
// total, k_scan_apply the prefix inside every chunk plus the chunk's offset.
constexpr int kScanChunk = 4 * kScanBlock;

// (with mdev: m = min(m, *mdev), the blocks taking the chunks in turn)
__global__ __launch_bounds__(kScanBlock) void k_scan_sums(const uint32_t* in, int64_t m, uint32_t* sums,
                                                           const unsigned long long* mdev = nullptr) {
    __shared__ unsigned long long ws[kScanBlock / 64];
    if (mdev) m = std::min<int64_t>(m, (int64_t)*mdev);
    const int64_t nb = (m + kScanChunk - 1) / kScanChunk;
    for (int64_t b = blockIdx.x; b < (mdev ? nb : (int64_t)blockIdx.x + 1); b += gridDim.x) {
        const int64_t i0 = b * kScanChunk + 4 * (int64_t)threadIdx.x;
        unsigned long long run = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) run += i0 + k < m ? (unsigned long long)in[i0 + k] : 0ull;
        run = pic::wave_sum(run);
        if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = run;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long t = 0;
            for (int q = 0; q < kScanBlock / 64; ++q) t += ws[q];
            sums[b] = (uint32_t)t;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_apply(const uint32_t* in, uint32_t* out, int64_t m,
                                                            const uint32_t* offs,
                                                            const unsigned long long* mdev = nullptr) {
    __shared__ unsigned long long wsum[kScanBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (mdev) m = std::min<int64_t>(m, (int64_t)*mdev);
    const int64_t nb = (m + kScanChunk - 1) / kScanChunk;
    for (int64_t b = blockIdx.x; b < (mdev ? nb : (int64_t)blockIdx.x + 1); b += gridDim.x) {
        const int64_t i0 = b * kScanChunk + 4 * (int64_t)threadIdx.x;
        unsigned long long v[4], run = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = i0 + k < m ? (unsigned long long)in[i0 + k] : 0ull;
            run += v[k];
        }
        unsigned long long x = run;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned long long y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        unsigned long long pre = offs[b];
        for (int q = 0; q < w; ++q) pre += wsum[q];
        pre += x - run;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (i0 + k < m) out[i0 + k] = (uint32_t)pre;
            pre += v[k];
        }
        __syncthreads();
    }
}

// zero the cell counts; the slots in use are the ones being grouped
__global__ void k_zero_u32(uint32_t* x, int64_t n, State* st) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0u;
    if (i == 0) {
        st->nbig = 0;
        st->nprod = 0;
        for (int s = 0; s < 3; ++s) st->ngrp[s] = st->n[s];
    }
}

struct CollArgs {
    Geo g;
    int64_t nc;        // cells (nr - 1) (nz - 1)
    double *r[3], *z[3], *vr[3], *vt[3], *vz[3];
    uint32_t* id[3];
    int64_t off[3];    // offset of each species in the per-slot work arrays
    int64_t cap[3];
    State* st;
    uint32_t* cnt;     // 3 nc particles per (species, cell)
    uint32_t* cpos;    // every slot's arrival order in its cell
    uint32_t* crank;   // every slot's rank (id order) in its cell
    uint32_t* start;   // 3 nc exclusive prefix of cnt
    uint32_t* seg;     // slots grouped by (species, cell), unordered within a cell
    uint32_t* segid;   // their ids
    uint32_t* sorted;  // the same, ascending id order within a cell
    uint32_t* big;     // keys of the cells above kRankSmall particles
    int32_t* cellof;   // cell of every slot (-1 free)
    uint8_t* used;     // the slot's particle had an event this step
    uint8_t* pflag;    // neutral slot: 1 impact ionization, 2 field ionization, 3 double ionization
    double* ve;        // neutral slot: the new electrons' velocities of an impact ionization (2 x 3)
    uint8_t* iflag;    // ion slot: 1 ionized to Cu2+ this step
    double* vei;       // ion slot: the new electron's velocity of that ionization
    uint8_t* charge;   // ion charge states (Cu2+ only)
    unsigned long long* pkey;  // product list: kind << 32 | id (kind 0 impact, 1 field, 2 Cu+ ionization)
    uint32_t* pslot;           // the neutral's (kinds 0, 1) or the ion's (kind 2) slot
    uint32_t *pci, *pce;       // per sorted entry: new ions, new electrons (0 beyond the list)
    uint32_t *ppi, *ppe;       // their exclusive prefixes
    int64_t pcap;              // cap[1] + cap[2], the longest list
    const double* E;
    const double* xs;
    int xs_n;
    double xs_emin, xs_lnr;
    double sig_max[3];  // per class: the largest tabulated sigma_el + sigma_iz (+ sigma_iz2), sigma_cx,
                        // sigma_izi (bounds)
    int cu2;
    double xi2;
    double h, dt, m_ion, xi;
    uint64_t seed;
    uint32_t step;
    double adk_c, adk_e, x32, dt_fs, ebsi;
    double e_min;  // [GV/m] below it w dt < 2^-60 (a draw is at least 2^-53): no field ionization
};

__device__ inline int cell_index(const Geo& g, double r, double z) {
    const int i = clampi((int)floor(r), 0, g.nr - 2), k = clampi((int)floor(z), 0, g.nz - 2);
    return k * (g.nr - 1) + i;
}

// cell of every slot in use, counts per (species, cell) and each particle's
// arrival place in its cell; clears the flags. Consecutive lanes of a
// wavefront in one cell (the common case after a reorder) take their places
// with one atomic for the run.
__global__ __launch_bounds__(kBlock) void k_cells(CollArgs a, int s) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = p < (int64_t)a.st->n[s];
    int32_t c = -1;
    if (in) {
        const uint32_t id = a.id[s][p];
        const double r = a.r[s][p], z = a.z[s][p];  // read with the id, not after it
        if (id != kDead) c = cell_index(a.g, r, z);
    }
    const int lane = threadIdx.x & 63;
    const int32_t prev = __shfl_up(c, 1, 64);
    const bool head = lane == 0 || prev != c;
    const uint64_t heads = __ballot(head);
    // the run of this lane: from its head (the highest head at or below it)
    // to the next head
    const uint64_t below = heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
    const int start = 63 - __builtin_clzll(below);
    const uint64_t above = lane == 63 ? 0ull : (heads >> (lane + 1));
    const int next = above ? lane + 1 + __builtin_ctzll(above) : 64;
    uint32_t base = 0;
    if (head && c >= 0) base = atomicAdd(&a.cnt[s * a.nc + c], (uint32_t)(next - lane));
    base = __shfl(base, start, 64);
    if (!in) return;
    if (c >= 0) a.cpos[a.off[s] + p] = base + (uint32_t)(lane - start);
    a.cellof[a.off[s] + p] = c;
    a.used[a.off[s] + p] = 0;
    if (s == 2) a.pflag[p] = 0;
    if (s == 1) a.iflag[p] = 0;
}

__global__ __launch_bounds__(kBlock) void k_place(CollArgs a, int s) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)a.st->n[s]) return;
    const int32_t c = a.cellof[a.off[s] + p];
    if (c < 0) return;
    const int64_t j = a.start[s * a.nc + c] + a.cpos[a.off[s] + p];
    a.seg[j] = (uint32_t)p;
    a.segid[j] = a.id[s][p];
}

// The deposit of the grouped electrons and ions in grouped order: the lanes
// of a wavefront that hold one cell add their node weights by a segmented
// sum over the lanes, and the first of them adds the sums to the cell's four
// nodes (integers, so the node charge does not depend on the order).
__global__ __launch_bounds__(kBlock) void k_deposit_grouped(CollArgs a, int64_t* rho) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = j < (int64_t)a.start[2 * a.nc];
    long long key = -1;
    long long w[4] = {0, 0, 0, 0};
    int64_t n0 = 0;
    if (act) {
        const int s = j < (int64_t)a.start[a.nc] ? 0 : 1;
        const uint32_t p = a.seg[j];
        const int32_t c = a.cellof[a.off[s] + p];
        key = (long long)s * a.nc + c;
        const Geo& g = a.g;
        const double R = a.r[s][p], Z = a.z[s][p];
        const int i = clampi((int)floor(R), 0, g.nr - 2), k = clampi((int)floor(Z), 0, g.nz - 2);
        const int64_t qr = pic::quantize(R - i, 20), qz = pic::quantize(Z - k, 20);
        const int64_t one = 1 << 20, sign = s == 0 ? -1 : (a.charge ? (int64_t)a.charge[p] : 1);
        n0 = (int64_t)k * g.nr + i;
        w[0] = sign * (one - qr) * (one - qz);
        w[1] = sign * qr * (one - qz);
        w[2] = sign * (one - qr) * qz;
        w[3] = sign * qr * qz;
    }
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const long long kk = __shfl_down(key, o, 64);
        const bool same = lane + o < 64 && kk == key;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const long long y = __shfl_down(w[t], o, 64);
            if (same) w[t] += y;
        }
    }
    const long long prev = __shfl_up(key, 1, 64);
    if (!act || (lane > 0 && prev == key)) return;
    unsigned long long* q = (unsigned long long*)rho;
    atomicAdd(q + n0, (unsigned long long)w[0]);
    atomicAdd(q + n0 + 1, (unsigned long long)w[1]);
    atomicAdd(q + n0 + a.g.nr, (unsigned long long)w[2]);
    atomicAdd(q + n0 + a.g.nr + 1, (unsigned long long)w[3]);
}

// Cells of up to kRankSmall particles of a species: each grouped particle's
// rank among its cell's particles (the number of smaller ids) is its place
// in ascending id order; the lanes of a wavefront that share a cell read the
// same addresses together. Larger cells are listed for k_sort_big.
__global__ __launch_bounds__(kBlock) void k_rank(CollArgs a) {
    // A cell of at most kRankSmall particles holding j lies within
    // kRankSmall - 1 places of j: the block's ids and that margin on each
    // side are staged in LDS once, and the counts read them there.
    __shared__ uint32_t sid[kBlock + 2 * kRankSmall];
    const int64_t j0 = (int64_t)blockIdx.x * kBlock, j = j0 + threadIdx.x;
    const int64_t total = a.st->total;  // the particles grouped, from the scan of the counts
    const int64_t w0 = j0 - kRankSmall;
    for (int q = threadIdx.x; q < kBlock + 2 * kRankSmall; q += kBlock) {
        const int64_t idx = w0 + q;
        sid[q] = idx >= 0 && idx < total ? a.segid[idx] : 0u;
    }
    __syncthreads();
    if (j >= total) return;
    const int s = j < (int64_t)a.start[a.nc] ? 0 : (j < (int64_t)a.start[2 * a.nc] ? 1 : 2);
    const uint32_t p = a.seg[j], myid = sid[j - w0];
    const int64_t key = s * a.nc + a.cellof[a.off[s] + p];
    const int64_t b = a.start[key], m = a.cnt[key];
    if (m > kRankSmall) {
        if (j == b) a.big[atomicAdd(&a.st->nbig, 1u)] = (uint32_t)key;
        return;
    }
    const uint32_t* ids = sid + (b - w0);
    int rank = 0;
    for (int k = 0; k < (int)m; ++k) rank += ids[k] < myid ? 1 : 0;
    a.sorted[b + rank] = p;
    a.crank[a.off[s] + p] = (uint32_t)rank;
}

// The listed cells, one per block in turn: up to kRankLds particles by a
// bitonic sort in LDS of id << 32 | slot (padded to a power of two with keys
// above every entry), beyond that by rank counting of the ids over LDS tiles
// of the cell (quadratic in the cell's particles).
__global__ __launch_bounds__(kBlock) void k_sort_big(CollArgs a) {
    __shared__ unsigned long long keys[kRankLds];
    const uint32_t nbig = a.st->nbig;
    for (uint32_t e = blockIdx.x; e < nbig; e += gridDim.x) {
        const int64_t key = a.big[e];
        const int64_t b = a.start[key], m = a.cnt[key];
        if (m <= kRankLds) {
            int P = 1;
            while (P < m) P <<= 1;
            for (int i = threadIdx.x; i < P; i += blockDim.x)
                keys[i] = i < m ? ((unsigned long long)a.segid[b + i] << 32 | a.seg[b + i]) : ~0ull;
            __syncthreads();
            for (int k = 2; k <= P; k <<= 1) {
                for (int jj = k >> 1; jj > 0; jj >>= 1) {
                    for (int i = threadIdx.x; i < P; i += blockDim.x) {
                        const int ixj = i ^ jj;
                        if (ixj > i) {
                            const unsigned long long x = keys[i], y = keys[ixj];
                            if ((x > y) == ((i & k) == 0)) {
                                keys[i] = y;
                                keys[ixj] = x;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            const int sp = (int)(key / a.nc);
            for (int i = threadIdx.x; i < m; i += blockDim.x) {
                const uint32_t slot = (uint32_t)(keys[i] & 0xFFFFFFFFull);
                a.sorted[b + i] = slot;
                a.crank[a.off[sp] + slot] = (uint32_t)i;
            }
            __syncthreads();  // keys are reused by the next cell
        } else {
            for (int64_t i0 = 0; i0 < m; i0 += blockDim.x) {
                const int64_t i = i0 + threadIdx.x;
                const uint32_t p = i < m ? a.seg[b + i] : 0xFFFFFFFFu;
                const unsigned long long myid = i < m ? a.segid[b + i] : ~0ull;
                int64_t rank = 0;
                for (int64_t t0 = 0; t0 < m; t0 += kRankLds) {
                    const int64_t tn = m - t0 < kRankLds ? m - t0 : kRankLds;
                    for (int64_t k = threadIdx.x; k < tn; k += blockDim.x) keys[k] = a.segid[b + t0 + k];
                    __syncthreads();
                    for (int64_t k = 0; k < tn; ++k) rank += keys[k] < myid ? 1 : 0;
                    __syncthreads();
                }
                if (i < m) {
                    a.sorted[b + rank] = p;
                    a.crank[a.off[key / a.nc] + p] = (uint32_t)rank;
                }
            }
        }
    }
}

__device__ inline double xs_at(const CollArgs& a, int k, double E) {
    const double* tab = a.xs + (int64_t)k * a.xs_n;
    const int n = a.xs_n;
    if (E <= a.xs_emin) return tab[0];
    if (E >= a.xs_emin * exp(a.xs_lnr)) return tab[n - 1];
    const double t = log(E / a.xs_emin) / a.xs_lnr * (double)(n - 1);
    int q = (int)floor(t);
    q = q > n - 2 ? n - 2 : (q < 0 ? 0 : q);
    const double f = t - q;
    return tab[q] + f * (tab[q + 1] - tab[q]);
}

__device__ inline void iso(double ct, double ph, double out[3]) {
    const double st = sqrt(1.0 - ct * ct);
    out[0] = st * cos(ph);
    out[1] = st * sin(ph);
    out[2] = ct;
}

// Pairs of class cls (1: e-Cu, 2: Cu+-Cu, 3: e-Cu+ with Cu2+), one thread
// per particle of the first species; each pair has one thread, so every
// particle is written by at most one thread of the class.
__global__ __launch_bounds__(kBlock) void k_pair(CollArgs a, int cls) {
    const int sa = cls == 2 ? 1 : 0;
    const int sb = cls == 3 ? 1 : 2;
    // one thread per grouped slot of the first species, in slot order (its
    // own reads and writes coalesce), with its rank in the cell
    const int64_t pa0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pa0 >= (int64_t)a.st->ngrp[sa]) return;
    const int32_t c = a.cellof[a.off[sa] + pa0];
    if (c < 0) return;
    const int64_t NA = a.cnt[sa * a.nc + c], NB = a.cnt[sb * a.nc + c];
    if (NB == 0) return;
    const int64_t qa = a.crank[a.off[sa] + pa0];
    const int64_t bB = a.start[sb * a.nc + c];
    const bool a_proj = NA <= NB;
    const int64_t NT = a_proj ? NB : NA;
    const uint32_t tag_pair = cls == 1 ? pic::kTagPair1 : (cls == 2 ? pic::kTagPair2 : kTagPairIon);
    const double uc = draw2(a.seed, (uint32_t)c, a.step, tag_pair, 0).a;
    int64_t shift = (int64_t)floor(uc * (double)NT);
    if (shift > NT - 1) shift = NT - 1;
    uint32_t pb;
    if (a_proj) {
        pb = a.sorted[bB + (shift + qa) % NT];
    } else {
        const int64_t q = (qa - shift + NA) % NA;
        if (q >= NB) return;
        pb = a.sorted[bB + q];
    }
    const uint32_t pa = (uint32_t)pa0;
    if (cls == 2 && a.used[a.off[2] + pb]) return;
    if (cls == 3 && (a.used[a.off[0] + pa] || a.used[a.off[1] + pb] || a.charge[pb] != 1)) return;
    const uint32_t pid = a_proj ? a.id[sa][pa] : a.id[sb][pb];
    const double h = a.h, dt = a.dt;
    double* AV[3] = {a.vr[sa], a.vt[sa], a.vz[sa]};
    double* BV[3] = {a.vr[sb], a.vt[sb], a.vz[sb]};
    const double vA[3] = {AV[0][pa], AV[1][pa], AV[2][pa]};
    const double vB[3] = {BV[0][pb], BV[1][pb], BV[2][pb]};
    const double u[3] = {(vA[0] - vB[0]) * h / dt, (vA[1] - vB[1]) * h / dt, (vA[2] - vB[2]) * h / dt};
    const double um = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const double ma = cls == 2 ? a.m_ion : kMe, mb = a.m_ion;
    const int i = c % (a.g.nr - 1);
    const double vol = kPi * (double)(2 * i + 1) * h * h * h;
    const double n = (double)NT / vol;
    const uint32_t tag = cls == 1 ? pic::kTagMcc1 : (cls == 2 ? pic::kTagMcc2 : kTagIon);
    const Draw2 d = draw2(a.seed, pid, a.step, tag, 0);
    // the largest cross section of the class bounds P from above: a draw at
    // or above that bound is no collision, without the table look-ups
    if (!(d.a < -expm1(-um * n * a.sig_max[cls - 1] * dt))) return;
    const double E = 0.5 * ma * um * um / kQe;
    double sig0, sig1 = 0.0, sig2 = 0.0;
    if (cls == 1) {
        sig0 = xs_at(a, 0, E);
        sig1 = E > a.xi ? xs_at(a, 1, E) : 0.0;
        if (a.cu2) sig2 = E > a.xi + a.xi2 ? xs_at(a, 3, E) : 0.0;
    } else if (cls == 2) {
        sig0 = xs_at(a, 2, E);
    } else {
        sig0 = E > a.xi2 ? xs_at(a, 4, E) : 0.0;
    }
    const double stot = a.cu2 && cls == 1 ? sig0 + sig1 + sig2 : sig0 + sig1;
    const double P = -expm1(-um * n * stot * dt);
    if (!(d.a < P)) return;
    int proc = 0;
    if (cls == 1) {
        if (d.b * stot < sig0) proc = 0;
        else if (!a.cu2 || d.b * stot < sig0 + sig1) proc = 1;
        else proc = 2;
    }
    a.used[a.off[sa] + pa] = 1;
    a.used[a.off[sb] + pb] = 1;
    if (cls == 2) {
        for (int k = 0; k < 3; ++k) {
            AV[k][pa] = vB[k];
            BV[k][pb] = vA[k];
        }
        atomicAdd(&a.st->events[3], 1ull);
        return;
    }
    if (cls == 1 && proc == 0) {
        // Eq. du: R^-1(theta, phi) [R^-1(theta', phi') - I] (0, 0, |u|)
        const Draw2 r = draw2(a.seed, pid, a.step, pic::kTagMcc1, 1);
        const double ct2 = 2.0 * r.a - 1.0, ph2 = 2.0 * kPi * r.b;
        const double up = sqrt(u[0] * u[0] + u[1] * u[1]);
        const double ct = u[2] / um, st = up / um;
        double cp = 1.0, sp = 0.0;
        if (up > 0.0) {
            cp = u[0] / up;
            sp = u[1] / up;
        }
        const double st2 = sqrt(1.0 - ct2 * ct2);
        const double w0 = um * st2 * cos(ph2), w1 = um * st2 * sin(ph2), w2 = um * (ct2 - 1.0);
        const double du[3] = {ct * cp * w0 - sp * w1 + st * cp * w2, ct * sp * w0 + cp * w1 + st * sp * w2,
                              -st * w0 + ct * w2};
        const double mu = ma * mb / (ma + mb);
        const double ka = mu / ma * dt / h, kb = mu / mb * dt / h;
        for (int k = 0; k < 3; ++k) {
            AV[k][pa] = vA[k] + ka * du[k];
            BV[k][pb] = vB[k] - kb * du[k];
        }
        atomicAdd(&a.st->events[1], 1ull);
        return;
    }
    // ionizations: in the frame of the neutral (or ion) the energy above the
    // threshold is shared by the electrons, each leaving isotropically
    const Draw2 r1 = draw2(a.seed, pid, a.step, tag, 1);
    const Draw2 r2 = draw2(a.seed, pid, a.step, tag, 2);
    const Draw2 r3 = draw2(a.seed, pid, a.step, tag, 3);
    double s1[3], s2[3];
    iso(2.0 * r1.a - 1.0, 2.0 * kPi * r1.b, s1);
    iso(2.0 * r2.a - 1.0, 2.0 * kPi * r2.b, s2);
    const double vn[3] = {vB[0] * h / dt, vB[1] * h / dt, vB[2] * h / dt};
    if (cls == 3) {
        // Cu+ + e -> Cu2+ + 2e above xi2; the ion keeps slot, id, velocity
        const double rest3 = E - a.xi2;
        const double g1 = r3.a * rest3, g2 = rest3 - g1;
        const double v1 = sqrt(2.0 * g1 * kQe / kMe), v2 = sqrt(2.0 * g2 * kQe / kMe);
        for (int k = 0; k < 3; ++k) {
            AV[k][pa] = (vn[k] + v1 * s1[k]) * dt / h;
            a.vei[3 * (int64_t)pb + k] = (vn[k] + v2 * s2[k]) * dt / h;
        }
        a.charge[pb] = 2;
        a.iflag[pb] = 1;
        atomicAdd(&a.st->events[6], 1ull);
        return;
    }
    if (proc == 1) {
        const double erem = E - a.xi;
        const double e1 = r3.a * erem, e2 = erem - e1;
        const double w1 = sqrt(2.0 * e1 * kQe / kMe), w2 = sqrt(2.0 * e2 * kQe / kMe);
        for (int k = 0; k < 3; ++k) {
            AV[k][pa] = (vn[k] + w1 * s1[k]) * dt / h;
            a.ve[6 * (int64_t)pb + k] = (vn[k] + w2 * s2[k]) * dt / h;
        }
        a.pflag[pb] = 1;
        atomicAdd(&a.st->events[2], 1ull);
        return;
    }
    // Cu + e -> Cu2+ + 3e above xi + xi2: shares U5, U6 (1 - U5) and the rest
    const Draw2 r4 = draw2(a.seed, pid, a.step, tag, 4);
    double s3[3];
    iso(2.0 * r4.a - 1.0, 2.0 * kPi * r4.b, s3);
    const double rest = E - a.xi - a.xi2;
    const double f1 = r3.a * rest, f2 = r3.b * (rest - f1), f3 = rest - f1 - f2;
    const double w1 = sqrt(2.0 * f1 * kQe / kMe), w2 = sqrt(2.0 * f2 * kQe / kMe), w3 = sqrt(2.0 * f3 * kQe / kMe);
    for (int k = 0; k < 3; ++k) {
        AV[k][pa] = (vn[k] + w1 * s1[k]) * dt / h;
        a.ve[6 * (int64_t)pb + k] = (vn[k] + w2 * s2[k]) * dt / h;
        a.ve[6 * (int64_t)pb + 3 + k] = (vn[k] + w3 * s3[k]) * dt / h;
    }
    a.pflag[pb] = 3;
    atomicAdd(&a.st->events[5], 1ull);
}

__device__ inline double bilinear(const Geo& g, const double* f, int stride, int comp, double r, double z) {
    const int i = clampi((int)floor(r), 0, g.nr - 2), k = clampi((int)floor(z), 0, g.nz - 2);
    const double fr = r - i, fz = z - k;
    const int64_t n = (int64_t)k * g.nr + i;
    return (1 - fr) * (1 - fz) * f[stride * n + comp] + fr * (1 - fz) * f[stride * (n + 1) + comp] +
           (1 - fr) * fz * f[stride * (n + g.nr) + comp] + fr * fz * f[stride * (n + g.nr + 1) + comp];
}

// Field ionization (Eq. dfi) of the neutrals without an event: rate per fs
// at the local field in GV/m, none above the barrier-suppression field.
__global__ __launch_bounds__(kBlock) void k_fi(CollArgs a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)a.st->n[2]) return;
    // the state read together (not after the id and flag tests)
    const uint32_t id = a.id[2][p];
    const uint8_t used = a.used[a.off[2] + p];
    const double R = a.r[2][p], Z = a.z[2][p];
    if (id == kDead || used) return;
    const double er = bilinear(a.g, a.E, 2, 0, R, Z);
    const double ez = bilinear(a.g, a.E, 2, 1, R, Z);
    const double Eg = sqrt(er * er + ez * ez) * 1e-9;
    // below e_min no draw can be smaller than w dt (the decision is the
    // formula's, without evaluating it)
    if (Eg > a.ebsi || !(Eg > a.e_min) || !(Eg > 0.0)) return;
    const double pdt = a.adk_c * pow(20.5 * a.x32 / Eg, a.adk_e) * exp(-6.83 * a.x32 / Eg) * a.dt_fs;
    if (pdt > draw2(a.seed, a.id[2][p], a.step, pic::kTagFi, 0).a) {
        a.pflag[p] = 2;
        a.used[a.off[2] + p] = 1;
        atomicAdd(&a.st->events[4], 1ull);
    }
}

// Products: impact ionizations (kind 0), field ionizations (kind 1), each by
// ascending neutral id, then ionizations of Cu+ (kind 2) by ascending ion
// id. The product entries are appended to a list (key kind << 32 | id, and
// the slot), the list is sorted by key, and exclusive prefixes of the new
// ions and electrons of the sorted entries give each product its slots and
// ids (ids in product order, the ion's first).
__global__ __launch_bounds__(kBlock) void k_prod_list(CollArgs a) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c2 = a.cap[2];
    bool put = false;
    unsigned long long key = 0;
    uint32_t slot = 0;
    if (e < c2) {
        if (e < (int64_t)a.st->n[2]) {
            const uint8_t f = a.pflag[e];
            if (f) {
                put = true;
                key = ((unsigned long long)(f == 2 ? 1 : 0) << 32) | a.id[2][e];
                slot = (uint32_t)e;
            }
        }
    } else if (e < c2 + a.cap[1]) {
        const int64_t p = e - c2;
        if (p < (int64_t)a.st->n[1] && a.iflag[p]) {
            put = true;
            key = (2ull << 32) | a.id[1][p];
            slot = (uint32_t)p;
        }
    }
    const unsigned long long q = pic::wave_append(&a.st->nprod, put);
    if (put) {
        a.pkey[q] = key;
        a.pslot[q] = slot;
    }
}

__device__ inline void pcmpx(unsigned long long* k, uint32_t* v, int64_t n, int64_t i, int64_t j) {
    if (j >= n) return;  // k[j] is +inf
    const unsigned long long x = k[i], y = k[j];
    if (x > y) {
        k[i] = y;
        k[j] = x;
        const uint32_t t = v[i];
        v[i] = v[j];
        v[j] = t;
    }
}

// Ascending sort of n keys with their values by one block: a bitonic network
// whose comparators all put the smaller key first (each merge starts with
// the mirrored pairs), so virtual +inf keys pad n to a power of two without
// being stored or moved.
__device__ inline void block_sort(unsigned long long* k, uint32_t* v, int64_t n) {
    int64_t P = 1;
    while (P < n) P <<= 1;
    for (int64_t kk = 2; kk <= P; kk <<= 1) {
        const int64_t hk = kk >> 1;
        for (int64_t t = threadIdx.x; t < P / 2; t += blockDim.x) {
            const int64_t base = (t / hk) * kk, r = t % hk;
            pcmpx(k, v, n, base + r, base + kk - 1 - r);
        }
        __syncthreads();
        for (int64_t j = hk >> 1; j > 0; j >>= 1) {
            for (int64_t t = threadIdx.x; t < P / 2; t += blockDim.x) {
                const int64_t i = (t / j) * 2 * j + t % j;
                pcmpx(k, v, n, i, i + j);
            }
            __syncthreads();
        }
    }
}

constexpr int kProdLds = 4096;  // product lists up to this long are sorted in LDS

__global__ __launch_bounds__(1024) void k_prod_sort(CollArgs a) {
    __shared__ unsigned long long lk[kProdLds];
    __shared__ uint32_t lv[kProdLds];
    const int64_t n = (int64_t)a.st->nprod;
    if (n <= 1) return;
    if (n <= kProdLds) {
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
            lk[i] = a.pkey[i];
            lv[i] = a.pslot[i];
        }
        __syncthreads();
        block_sort(lk, lv, n);
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
            a.pkey[i] = lk[i];
            a.pslot[i] = lv[i];
        }
    } else {
        block_sort(a.pkey, a.pslot, n);  // in global memory, the block's own
    }
}

// new ions and electrons of every sorted entry (grid-stride over the list)
__global__ __launch_bounds__(kBlock) void k_prod_counts(CollArgs a) {
    const int64_t n = (int64_t)a.st->nprod;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t kind = (uint32_t)(a.pkey[j] >> 32);
        uint32_t ni = 0, ne = 1;
        if (kind == 0) {
            ni = 1;
            ne = a.pflag[a.pslot[j]] == 3 ? 2 : 1;
        } else if (kind == 1) {
            ni = 1;
        }
        a.pci[j] = ni;
        a.pce[j] = ne;
    }
}

// room for the products' ions and electrons and their ids
__global__ void k_prod_commit(CollArgs a) {
    if (threadIdx.x != 0) return;
    State* st = a.st;
    st->skip = 0;
    const int64_t L = (int64_t)st->nprod;
    const unsigned long long TI = L ? (unsigned long long)a.ppi[L - 1] + a.pci[L - 1] : 0ull;
    const unsigned long long TE = L ? (unsigned long long)a.ppe[L - 1] + a.pce[L - 1] : 0ull;
    if (TI + TE == 0) return;
    if (st->n[0] + TE > (unsigned long long)a.cap[0] || st->n[1] + TI > (unsigned long long)a.cap[1]) {
        st->skip = 1;
        if (st->error == 0) st->error = PIC_E_CAPACITY;
        return;
    }
    if (st->next_id + TI + TE > (unsigned long long)kDead) {
        st->skip = 1;
        if (st->error == 0) st->error = PIC_E_OVERFLOW;
        return;
    }
    st->base_n[0] = st->n[0];
    st->base_n[1] = st->n[1];
    st->base_id = st->next_id;
    st->n[0] += TE;
    st->n[1] += TI;
    st->next_id += TI + TE;
}

// the slots and ids of sorted entry j
__device__ inline void prod_place_one(const CollArgs& a, int64_t j) {
    const uint32_t kind = (uint32_t)(a.pkey[j] >> 32);
    const int64_t p = a.pslot[j];
    const uint32_t ne = a.pce[j];
    const uint64_t oi = a.ppi[j], oe = a.ppe[j];
    const uint64_t id0 = a.st->base_id + oi + oe;
    const uint64_t se = a.st->base_n[0] + oe;
    if (kind == 2) {
        // ionization of Cu+: one electron at the ion
        a.r[0][se] = a.r[1][p];
        a.z[0][se] = a.z[1][p];
        a.vr[0][se] = a.vei[3 * p];
        a.vt[0][se] = a.vei[3 * p + 1];
        a.vz[0][se] = a.vei[3 * p + 2];
        a.id[0][se] = (uint32_t)id0;
        return;
    }
    const uint8_t f = a.pflag[p];
    const uint64_t si = a.st->base_n[1] + oi;
    a.r[1][si] = a.r[2][p];
    a.z[1][si] = a.z[2][p];
    a.vr[1][si] = a.vr[2][p];
    a.vt[1][si] = a.vt[2][p];
    a.vz[1][si] = a.vz[2][p];
    a.id[1][si] = (uint32_t)id0;
    if (a.charge) a.charge[si] = f == 3 ? 2 : 1;
    for (uint32_t q = 0; q < ne; ++q) {
        a.r[0][se + q] = a.r[2][p];
        a.z[0][se + q] = a.z[2][p];
        if (f == 2) {
            a.vr[0][se + q] = a.vr[2][p];
            a.vt[0][se + q] = a.vt[2][p];
            a.vz[0][se + q] = a.vz[2][p];
        } else {
            a.vr[0][se + q] = a.ve[6 * p + 3 * q];
            a.vt[0][se + q] = a.ve[6 * p + 3 * q + 1];
            a.vz[0][se + q] = a.ve[6 * p + 3 * q + 2];
        }
        a.id[0][se + q] = (uint32_t)(id0 + 1 + q);
    }
    a.id[2][p] = kDead;
}

__global__ __launch_bounds__(kBlock) void k_prod_place(CollArgs a) {
    if (a.st->skip) return;
    const int64_t n = (int64_t)a.st->nprod;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        prod_place_one(a, j);
}

// Reorder of species s by cell, ascending id in a cell (the grouping's
// order), freed slots dropped: into the work copies, then back.
struct ReorderArgs {
    double *r, *z, *vr, *vt, *vz;
    uint32_t* id;
    uint8_t* charge;
    double *tr, *tz, *tvr, *tvt, *tvz;
    uint32_t* tid;
    uint8_t* tcharge;
    const uint32_t* sorted;
    const uint32_t* start;  // of the species' first cell; the next species' start, or total
    int64_t first, next;    // indices into start (next < 0: the grouped total)
    State* st;
};

__device__ inline int64_t reorder_count(const ReorderArgs& a) {
    const int64_t b = a.start[a.first];
    const int64_t e = a.next >= 0 ? (int64_t)a.start[a.next] : (int64_t)a.st->total;
    return e - b;
}

__global__ __launch_bounds__(kBlock) void k_reorder_gather(ReorderArgs a) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= reorder_count(a)) return;
    const uint32_t p = a.sorted[a.start[a.first] + j];
    a.tr[j] = a.r[p];
    a.tz[j] = a.z[p];
    a.tvr[j] = a.vr[p];
    a.tvt[j] = a.vt[p];
    a.tvz[j] = a.vz[p];
    a.tid[j] = a.id[p];
    if (a.charge) a.tcharge[j] = a.charge[p];
}

__global__ __launch_bounds__(kBlock) void k_reorder_back(ReorderArgs a, int sp) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = reorder_count(a);
    if (j == 0) a.st->n[sp] = (unsigned long long)n;
    if (j >= n) return;
    a.r[j] = a.tr[j];
    a.z[j] = a.tz[j];
    a.vr[j] = a.tvr[j];
    a.vt[j] = a.tvt[j];
    a.vz[j] = a.tvz[j];
    a.id[j] = a.tid[j];
    if (a.charge) a.charge[j] = a.tcharge[j];
}

// room for the T = st->total emitted electrons and their ids
__global__ void k_emit_commit(State* st, int64_t cap0) {
    if (threadIdx.x != 0) return;
    const unsigned long long T = st->total;
    st->skip = 0;
    if (T == 0) return;
    if (st->n[0] + T > (unsigned long long)cap0) {
        st->skip = 1;
        if (st->error == 0) st->error = PIC_E_CAPACITY;
        return;
    }
    if (st->next_id + T > (unsigned long long)kDead) {
        st->skip = 1;
        if (st->error == 0) st->error = PIC_E_OVERFLOW;
        return;
    }
    st->base_n[0] = st->n[0];
    st->base_id = st->next_id;
    st->n[0] += T;
    st->next_id += T;
    st->injected += T;
}

// ---------------------------------------------------------------------------
// Field emission from rings of the tip surface
struct EmitArgs {
    Geo g;
    const double* phi;
    int rings;
    int64_t npatch;
    double h, dt, phi_w, phi_w15, fn_a, fn_b, fn_cs2;
    uint64_t seed;
    uint32_t step;
    int64_t cap0;
    uint32_t* cnt;    // electrons of each patch
    uint64_t* offs;   // their exclusive prefix
    double *r, *z, *vr, *vt, *vz;
    uint32_t* id;
    State* st;
};

// point of patch p at the ring parameter ua: {r, z, n_r, n_z, area}
__device__ inline void ring_point(const EmitArgs& a, int64_t p, double ua, double out[5]) {
    const double R = a.g.R, zc = a.g.H - a.g.R;
    if (p < a.rings) {
        const double ct = 1.0 - ((double)p + ua) / (double)a.rings;
        const double st = sqrt(1.0 - ct * ct);
        out[0] = R * st;
        out[1] = zc + R * ct;
        out[2] = st;
        out[3] = ct;
        out[4] = 2.0 * kPi * R * R / (double)a.rings;
    } else {
        const int64_t q = p - a.rings;
        const double zlo = (double)q, zhi = fmin((double)(q + 1), zc);
        out[0] = R;
        out[1] = zlo + ua * (zhi - zlo);
        out[2] = 1.0;
        out[3] = 0.0;
        out[4] = 2.0 * kPi * R * (zhi - zlo);
    }
}

__global__ __launch_bounds__(kBlock) void k_emit_count(EmitArgs a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.npatch) return;
    double q[5];
    ring_point(a, p, 0.5, q);
    const double F = bilinear(a.g, a.phi, 1, 0, q[0] + q[2], q[1] + q[3]) / a.h;
    double J = 0.0;
    if (F > 0.0) {
        double f = a.fn_cs2 * F / (a.phi_w * a.phi_w);
        if (f > 1.0) f = 1.0;
        const double lf = log(f);
        const double v = 1.0 - f + (f / 6.0) * lf;
        const double t = 1.0 + f / 9.0 - (f / 18.0) * lf;
        J = a.fn_a * F * F / (a.phi_w * t * t) * exp(-v * a.fn_b * a.phi_w15 / F);
    }
    const double N = J * q[4] * a.h * a.h * a.dt / kQe;
    const double fl = floor(N);
    // beyond the capacity the count only has to overflow it
    const double lim = (double)a.cap0 + 1.0;
    int64_t k = fl < lim ? (int64_t)fl : (int64_t)lim;
    if (draw2(a.seed, (uint32_t)p, a.step, pic::kTagInj, 0).a < N - fl) ++k;
    a.cnt[p] = (uint32_t)(k < (int64_t)a.cap0 + 1 ? k : (int64_t)a.cap0 + 1);
}

// one block per patch, its electrons in order
__global__ __launch_bounds__(kBlock) void k_emit_place(EmitArgs a) {
    const int64_t p = blockIdx.x;
    if (p >= a.npatch || a.st->skip) return;
    const uint32_t k = a.cnt[p];
    for (uint32_t j = threadIdx.x; j < k; j += blockDim.x) {
        const double ua = draw2(a.seed, (uint32_t)p, a.step, pic::kTagInj, 1u + j).a;
        double q[5];
        ring_point(a, p, ua, q);
        const uint64_t o = a.offs[p] + j;
        const uint64_t s = a.st->base_n[0] + o;
        a.r[s] = q[0] + 1e-3 * q[2];
        a.z[s] = q[1] + 1e-3 * q[3];
        a.vr[s] = 0.0;
        a.vt[s] = 0.0;
        a.vz[s] = 0.0;
        a.id[s] = (uint32_t)(a.st->base_id + o);
    }
}

__global__ void k_mg_types(Lv F, int cnr, int cnz, int sr, int sz, uint8_t* tc) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (int64_t)cnr * cnz) return;
    const int I = (int)(n % cnr), K = (int)(n / cnr);
    tc[n] = F.type[(int64_t)(sz * K) * F.nr + sr * I] == kFree ? kFree : kHeld0;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// the multigrid levels of a grid: dims and coupling factors
struct MgDims {
    int levels;
    int nr[kMgMaxLevels], nz[kMgMaxLevels], sr[kMgMaxLevels], sz[kMgMaxLevels];  // sr, sz: halved to level l + 1
    double fr[kMgMaxLevels], fa[kMgMaxLevels];
};

MgDims mg_dims(int nr, int nz) {
    MgDims d{};
    int a = 0, b = 0;
    d.levels = 1;
    d.nr[0] = nr;
    d.nz[0] = nz;
    d.fr[0] = d.fa[0] = 1.0;
    for (int l = 0; l + 1 < kMgMaxLevels; ++l) {
        if ((int64_t)d.nr[l] * d.nz[l] <= kMgDirectMax) break;  // solved directly
        const bool hr = (d.nr[l] - 1) % 2 == 0 && d.nr[l] - 1 >= 4;
        const bool hz = (d.nz[l] - 1) % 2 == 0 && d.nz[l] - 1 >= 4;
        if (!hr && !hz) break;
        d.sr[l] = hr ? 2 : 1;
        d.sz[l] = hz ? 2 : 1;
        a += hr ? 1 : 0;
        b += hz ? 1 : 0;
        d.nr[l + 1] = hr ? (d.nr[l] - 1) / 2 + 1 : d.nr[l];
        d.nz[l + 1] = hz ? (d.nz[l] - 1) / 2 + 1 : d.nz[l];
        d.fr[l + 1] = std::ldexp(1.0, b);
        d.fa[l + 1] = std::ldexp(1.0, 2 * a - b);
        d.levels = l + 2;
    }
    return d;
}

int64_t patches(const pic_rz_config* c) {
    if (c->fn_rings <= 0) return 0;
    const double zc = (c->tip_h - c->tip_r) / c->h;
    return (int64_t)c->fn_rings + (zc > 0.0 ? (int64_t)std::ceil(zc) : 0);
}

// work memory carved from the scratch buffer
struct Work {
    State* st = nullptr;
    double *r = nullptr, *p = nullptr, *q = nullptr, *part = nullptr;  // CG
    unsigned long long* cnt = nullptr;                                   // moments counters (8)
    uint32_t *ccnt = nullptr, *start = nullptr;                          // 3 nc each
    uint32_t *cpos = nullptr, *crank = nullptr;                          // sum of caps each
    uint32_t *ssum = nullptr, *spre = nullptr;                           // chunk sums of the scans
    uint32_t *seg = nullptr, *segid = nullptr, *sorted = nullptr;        // sum of caps each
    uint32_t* big = nullptr;                                             // 3 nc
    int32_t* cellof = nullptr;
    uint8_t* used = nullptr;
    uint8_t* pflag = nullptr;  // cap[2]
    double* ve = nullptr;      // 6 cap[2]
    uint8_t* iflag = nullptr;  // cap[1]
    double* vei = nullptr;     // 3 cap[1]
    unsigned long long* pkey = nullptr;         // cap[1] + cap[2]
    uint32_t* pslot = nullptr;
    uint32_t *pci = nullptr, *pce = nullptr, *ppi = nullptr, *ppe = nullptr;  // cap[1] + cap[2] each
    // reorder work copies of one species (the largest capacity)
    double *tr = nullptr, *tz = nullptr, *tvr = nullptr, *tvt = nullptr, *tvz = nullptr;
    uint32_t* tid = nullptr;
    uint8_t* tcharge = nullptr;
    uint32_t* pcnt = nullptr;                   // patches
    uint64_t* poff = nullptr;
    double* z = nullptr;                        // preconditioned residual (nodes)
    // multigrid levels: types (level 0: the node types), two iterates, the
    // right-hand side (level 0: the CG residual) and the residual
    uint8_t* mtype[kMgMaxLevels] = {};
    double *mxa[kMgMaxLevels] = {}, *mxb[kMgMaxLevels] = {}, *mb[kMgMaxLevels] = {};
    double* minv = nullptr;  // inverse of the coarsest operator (kMgDirectMax^2)
    double* phi_prev = nullptr;  // the previous step potential (the guess's extrapolation)
};

size_t layout(const pic_rz_config* c, const int64_t cap[3], char* base, Work* w) {
    const size_t nn = (size_t)c->nr * c->nz;
    const size_t nc = (size_t)(c->nr - 1) * (c->nz - 1);
    const size_t ncap = (size_t)(cap[0] + cap[1] + cap[2]);
    const size_t nprod = (size_t)(cap[2] + cap[1]);
    const size_t capmax = (size_t)std::max(cap[0], std::max(cap[1], cap[2]));
    const size_t np = (size_t)patches(c);
    size_t off = 0;
    auto take = [&](size_t b) -> char* {
        char* x = base ? base + off : nullptr;
        off = align256(off + b);
        return x;
    };
    Work t;
    t.st = (State*)take(sizeof(State));
    t.r = (double*)take(nn * 8);
    t.p = (double*)take(nn * 8);
    t.q = (double*)take(nn * 8);
    t.part = (double*)take(4 * kCgBlocks * 8);
    t.cnt = (unsigned long long*)take(8 * 8);
    t.ccnt = (uint32_t*)take(3 * nc * 4);
    t.start = (uint32_t*)take(3 * nc * 4);
    t.cpos = (uint32_t*)take(ncap * 4);
    t.crank = (uint32_t*)take(ncap * 4);
    const size_t nscan = std::max(3 * nc, nprod) / kScanChunk + 2;
    t.ssum = (uint32_t*)take(nscan * 4);
    t.spre = (uint32_t*)take(nscan * 4);
    t.seg = (uint32_t*)take(ncap * 4);
    t.segid = (uint32_t*)take(ncap * 4);
    t.sorted = (uint32_t*)take(ncap * 4);
    t.big = (uint32_t*)take(3 * nc * 4);
    t.cellof = (int32_t*)take(ncap * 4);
    t.used = (uint8_t*)take(ncap);
    t.pflag = (uint8_t*)take((size_t)cap[2]);
    t.ve = (double*)take((size_t)cap[2] * 48);
    t.iflag = (uint8_t*)take((size_t)cap[1]);
    t.vei = (double*)take((size_t)cap[1] * 24);
    t.pkey = (unsigned long long*)take(nprod * 8 + 8);
    t.pslot = (uint32_t*)take(nprod * 4 + 4);
    t.tr = (double*)take(capmax * 8);
    t.tz = (double*)take(capmax * 8);
    t.tvr = (double*)take(capmax * 8);
    t.tvt = (double*)take(capmax * 8);
    t.tvz = (double*)take(capmax * 8);
    t.tid = (uint32_t*)take(capmax * 4);
    t.tcharge = (uint8_t*)take(capmax);
    t.pci = (uint32_t*)take(nprod * 4 + 4);
    t.pce = (uint32_t*)take(nprod * 4 + 4);
    t.ppi = (uint32_t*)take(nprod * 4 + 4);
    t.ppe = (uint32_t*)take(nprod * 4 + 4);
    t.pcnt = (uint32_t*)take(np * 4 + 4);
    t.poff = (uint64_t*)take(np * 8 + 8);
    t.z = (double*)take(nn * 8);
    const MgDims d = mg_dims(c->nr, c->nz);
    for (int l = 0; l < d.levels; ++l) {
        const size_t m = (size_t)d.nr[l] * d.nz[l];
        if (l > 0) {
            t.mtype[l] = (uint8_t*)take(m);
            t.mb[l] = (double*)take(m * 8);
        }
        t.mxa[l] = (double*)take(m * 8);
        t.mxb[l] = l == 0 ? t.z : (double*)take(m * 8);
    }
    t.minv = (double*)take((size_t)kMgDirectMax * kMgDirectMax * 8);
    t.phi_prev = (double*)take(nn * 8);
    if (w) *w = t;
    return off + 256;
}

const char* check(const pic_rz_config* c) {
    if (!c) return "config is NULL";
    if (c->nr < 4 || c->nz < 4) return "nr, nz must be >= 4";
    if ((int64_t)c->nr * c->nz >= (int64_t)1 << 31) return "grid too large";
    if (!(c->h > 0) || !(c->dt > 0)) return "h and dt must be positive";
    if (!(c->tip_r >= 0) || !(c->tip_h >= c->tip_r)) return "need tip_r >= 0 and tip_h >= tip_r";
    if (c->tip_h / c->h + 2.0 >= c->nz - 1 || c->tip_r / c->h + 2.0 >= c->nr - 1)
        return "the tip does not fit in the box with two spacings to spare";
    if (!(c->m_ion > 0)) return "m_ion must be positive";
    if (!(c->laplace_rtol > 0) || !(c->step_rtol > 0) || c->maxit < 1) return "need positive tolerances and maxit";
    if (c->xs_n < 0 || c->xs_n == 1) return "xs_n must be 0 or >= 2";
    if (c->xs_n > 0 && !(c->xs_emin > 0 && c->xs_emax > c->xs_emin && c->xi > 0))
        return "collisions need 0 < xs_emin < xs_emax and xi > 0";
    if (c->fn_rings < 0 || c->fn_rings > (1 << 20)) return "fn_rings out of range";
    if (c->cu2 != 0 && c->cu2 != 1) return "cu2 must be 0 or 1";
    if (c->sort_every < 0) return "sort_every must be >= 0";
    if (c->cu2 && !(c->xs_n > 0 && c->xi2 > 0)) return "Cu2+ needs the five tables and xi2 > 0";
    if (c->fn_rings > 0 && !(c->phi_w > 0 && c->tip_r > 0)) return "emission needs phi_w > 0 and a tip";
    return nullptr;
}

bool caps_ok(const int64_t cap[3]) {
    for (int s = 0; s < 3; ++s)
        if (cap[s] < 0 || cap[s] >= ((int64_t)1 << 31)) return false;
    return cap[0] + cap[1] + cap[2] < ((int64_t)1 << 32);
}

}  // namespace pic_rz

struct pic_rz_ctx {
    pic_rz_config cfg;
    pic_rz_buffers buf;
    hipStream_t stream = nullptr;
    pic_rz::Geo g;
    pic_rz::Work w;
    pic_rz::MgDims mg;
    pic_rz::State* st = nullptr;
    double *r = nullptr, *p = nullptr, *q = nullptr, *part = nullptr;
    unsigned long long* cnt = nullptr;
    double V0 = 0.0, F1 = 0.0;
    int64_t step = 0;
    int last_iters = 0;
    double sig_max[3] = {0.0, 0.0, 0.0};  // bounds of the class cross sections, from the tables
    const double* mg_inv = nullptr;        // inverse of the coarsest multigrid operator (w.minv), or null
    int n_prev = 0;                        // step potentials recorded for the guess (0, 1, 2)
    // two PCG iterations of the step solve (phi = buf.phi) as one graph
    hipStream_t cap_stream = nullptr;
    hipGraph_t pcg_graph = nullptr;
    hipGraphExec_t pcg_exec = nullptr;
    ~pic_rz_ctx() {
        if (pcg_exec) (void)hipGraphExecDestroy(pcg_exec);
        if (pcg_graph) (void)hipGraphDestroy(pcg_graph);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
    std::string err;
};

namespace {

using namespace pic_rz;

pic_status fail(pic_rz_ctx* c, pic_status s, const std::string& m) {
    if (c) c->err = m;
    return s;
}

pic_status hip_ok(pic_rz_ctx* c, hipError_t e, const char* what) {
    if (e == hipSuccess) return PIC_OK;
    return fail(c, PIC_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

unsigned grid_of(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kBlock - 1) / kBlock); }

CgArgs cg_args(pic_rz_ctx* c, double* phi, double V0) {
    CgArgs a;
    a.g = c->g;
    a.type = c->buf.node_type;
    a.rho = c->buf.rho;
    a.phi = phi;
    a.r = c->r;
    a.p = c->p;
    a.q = c->q;
    a.z = c->w.z;
    a.part = c->part;
    a.st = c->st;
    a.qscale = std::ldexp(1.0, -40) * kQe / (kPi * kEps0 * c->cfg.h);
    a.V0 = V0;
    return a;
}

Lv level(const pic_rz_ctx* c, int l) {
    Lv L;
    L.nr = c->mg.nr[l];
    L.nz = c->mg.nz[l];
    L.fr = c->mg.fr[l];
    L.fa = c->mg.fa[l];
    L.type = l == 0 ? c->buf.node_type : c->w.mtype[l];
    return L;
}

unsigned mg_grid(const Lv& L) {
    const int64_t nn = (int64_t)L.nr * L.nz;
    return (unsigned)std::min<int64_t>(1 << 14, std::max<int64_t>(1, (nn + kBlock - 1) / kBlock));  // a node a thread
}

// x_b = M b on level l (a V-cycle below it); x_a is work space
void vcycle(pic_rz_ctx* c, int l, const double* b, double* xa, double* xb) {
    const Lv L = level(c, l);
    const unsigned G = mg_grid(L);
    const State* st = c->st;
    int64_t below = 0;  // nodes of the levels from l down
    for (int k = l; k < c->mg.levels; ++k) below += (int64_t)c->mg.nr[k] * c->mg.nz[k];
    if (below <= kMgLdsNodes && l < c->mg.levels - 1) {
        MgLds m{};
        m.l0 = l;
        m.levels = c->mg.levels;
        int off = 0;
        for (int k = l; k < c->mg.levels; ++k) {
            m.lv[k] = level(c, k);
            m.off[k] = off;
            off += c->mg.nr[k] * c->mg.nz[k];
            m.sr[k] = c->mg.sr[k];
            m.sz[k] = c->mg.sz[k];
        }
        m.b = b;
        m.x = xb;
        m.inv = c->mg_inv;
        hipLaunchKernelGGL(k_mg_lds, dim3(1), dim3(kMgLdsBlock), 0, c->stream, m, st);
        return;
    }
    if (l == c->mg.levels - 1) {
        if ((int64_t)L.nr * L.nz <= kMgCoarseMax) {
            hipLaunchKernelGGL(k_mg_coarse, dim3(1), dim3(kBlock), 0, c->stream, L, b, xb, c->mg_inv, st);
        } else {
            hipLaunchKernelGGL(k_mg_jacobi, dim3(G), dim3(kBlock), 0, c->stream, L, (const double*)xb, xa, b, 1, st);
            hipLaunchKernelGGL(k_mg_jacobi, dim3(G), dim3(kBlock), 0, c->stream, L, (const double*)xa, xb, b, 0, st);
            hipLaunchKernelGGL(k_mg_jacobi, dim3(G), dim3(kBlock), 0, c->stream, L, (const double*)xb, xa, b, 0, st);
            hipLaunchKernelGGL(k_mg_jacobi, dim3(G), dim3(kBlock), 0, c->stream, L, (const double*)xa, xb, b, 0, st);
        }
        return;
    }
    const Lv Cl = level(c, l + 1);
    const int sr = c->mg.sr[l], sz = c->mg.sz[l];
    // two sweeps from zero, the residual restricted, the coarse correction,
    // two sweeps (the first with the correction formed on the fly)
    // (sr, sz) is (2, 2), (2, 1) or (1, 2): a level is made only where a dimension halves
    auto resid_restrict = sr == 2 ? (sz == 2 ? k_mg_resid_restrict<2, 2> : k_mg_resid_restrict<2, 1>)
                                  : k_mg_resid_restrict<1, 2>;
    auto prolong_smooth = sr == 2 ? (sz == 2 ? k_mg_prolong_smooth<2, 2> : k_mg_prolong_smooth<2, 1>)
                                  : k_mg_prolong_smooth<1, 2>;
    hipLaunchKernelGGL(k_mg_smooth2, dim3(G), dim3(kBlock), 0, c->stream, L, b, xb, st);
    hipLaunchKernelGGL(resid_restrict, dim3(mg_grid(Cl)), dim3(kBlock), 0, c->stream, L, Cl, (const double*)xb, b,
                       c->w.mb[l + 1], st);
    vcycle(c, l + 1, c->w.mb[l + 1], c->w.mxa[l + 1], c->w.mxb[l + 1]);
    hipLaunchKernelGGL(prolong_smooth, dim3(G), dim3(kBlock), 0, c->stream, L, Cl, (const double*)c->w.mxb[l + 1],
                       (const double*)xb, xa, b, st);
    hipLaunchKernelGGL(k_mg_jacobi, dim3(G), dim3(kBlock), 0, c->stream, L, (const double*)xa, xb, b, 0, st);
}

// The inverse of the coarsest multigrid operator, when that level has at most
// kMgDirectMax nodes: the operator of lv_apply over the free nodes (held ones
// at zero), inverted on the host by Gauss-Jordan elimination with partial
// pivoting, stored nc x nc with zero rows and columns at held nodes.
pic_status mg_inverse(pic_rz_ctx* c) {
    c->mg_inv = nullptr;
    const int l = c->mg.levels - 1;
    const int nr = c->mg.nr[l], nz = c->mg.nz[l], nc = nr * nz;
    if (nc > kMgDirectMax) return PIC_OK;
    std::vector<uint8_t> ty((size_t)nc);
    const uint8_t* dty = l == 0 ? c->buf.node_type : c->w.mtype[l];
    pic_status s = hip_ok(c, hipMemcpyAsync(ty.data(), dty, (size_t)nc, hipMemcpyDeviceToHost, c->stream), "copy");
    if (s == PIC_OK) s = hip_ok(c, hipStreamSynchronize(c->stream), "sync");
    if (s != PIC_OK) return s;
    std::vector<int> fr;  // free nodes
    std::vector<int> at((size_t)nc, -1);
    for (int n = 0; n < nc; ++n)
        if (ty[(size_t)n] == kFree) {
            at[(size_t)n] = (int)fr.size();
            fr.push_back(n);
        }
    const int nf = (int)fr.size();
    std::vector<double> a((size_t)nf * nf, 0.0), v((size_t)nf * nf, 0.0);
    for (int r = 0; r < nf; ++r) {
        const int n = fr[(size_t)r], i = n % nr, k = n / nr;
        const double cin = i > 0 ? c->mg.fr[l] * 2.0 * (i - 0.5) : 0.0;
        const double cout = i < nr - 1 ? c->mg.fr[l] * 2.0 * (i + 0.5) : 0.0;
        const double hi = std::min(i + 0.5, nr - 1.0), lo = std::max(i - 0.5, 0.0);
        const double cax = c->mg.fa[l] * (hi * hi - lo * lo);
        a[(size_t)r * nf + r] = cin + cout + 2.0 * cax;
        auto off = [&](int m, double cf) {
            if (cf != 0.0 && at[(size_t)m] >= 0) a[(size_t)r * nf + at[(size_t)m]] -= cf;
        };
        if (i > 0) off(n - 1, cin);
        if (i < nr - 1) off(n + 1, cout);
        if (k > 0) off(n - nr, cax);
        if (k < nz - 1) off(n + nr, cax);
        v[(size_t)r * nf + r] = 1.0;
    }
    for (int col = 0; col < nf; ++col) {
        int piv = col;
        for (int r = col + 1; r < nf; ++r)
            if (std::fabs(a[(size_t)r * nf + col]) > std::fabs(a[(size_t)piv * nf + col])) piv = r;
        if (!(std::fabs(a[(size_t)piv * nf + col]) > 0.0))
            return fail(c, PIC_E_INVALID_ARG, "the coarsest multigrid operator is singular");
        if (piv != col)
            for (int j = 0; j < nf; ++j) {
                std::swap(a[(size_t)piv * nf + j], a[(size_t)col * nf + j]);
                std::swap(v[(size_t)piv * nf + j], v[(size_t)col * nf + j]);
            }
        const double d = a[(size_t)col * nf + col];
        for (int j = 0; j < nf; ++j) {
            a[(size_t)col * nf + j] /= d;
            v[(size_t)col * nf + j] /= d;
        }
        for (int r = 0; r < nf; ++r) {
            if (r == col) continue;
            const double f = a[(size_t)r * nf + col];
            if (f == 0.0) continue;
            for (int j = 0; j < nf; ++j) {
                a[(size_t)r * nf + j] -= f * a[(size_t)col * nf + j];
                v[(size_t)r * nf + j] -= f * v[(size_t)col * nf + j];
            }
        }
    }
    std::vector<double> inv((size_t)nc * nc, 0.0);
    for (int r = 0; r < nf; ++r)
        for (int q = 0; q < nf; ++q) inv[(size_t)fr[(size_t)r] * nc + fr[(size_t)q]] = v[(size_t)r * nf + q];
    s = hip_ok(c, hipMemcpyAsync(c->w.minv, inv.data(), inv.size() * 8, hipMemcpyHostToDevice, c->stream), "copy");
    if (s == PIC_OK) s = hip_ok(c, hipStreamSynchronize(c->stream), "sync");
    if (s == PIC_OK) c->mg_inv = c->w.minv;
    return s;
}

// Multigrid-preconditioned CG from the current phi (held nodes set to 0 /
// V0); without charge the q vector, zeroed, stands for the charge (it is read
// only by k_cg_init, before the iterations use q)
pic_status cg(pic_rz_ctx* c, double* phi, double V0, bool with_charge, double rtol, int maxit, int* iters) {
    CgArgs a = cg_args(c, phi, V0);
    if (!with_charge) {
        pic_status s = hip_ok(c, hipMemsetAsync(c->q, 0, (size_t)c->g.nr * c->g.nz * 8, c->stream), "zero");
        if (s != PIC_OK) return s;
        a.rho = (const int64_t*)c->q;
    }
    hipLaunchKernelGGL(k_cg_init, dim3(kCgBlocks), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(64), 0, c->stream, a, rtol, maxit);
    vcycle(c, 0, c->r, c->w.mxa[0], c->w.z);
    hipLaunchKernelGGL(k_pcg_rz, dim3(kCgBlocks), dim3(kBlock), 0, c->stream, a, 1);
    hipLaunchKernelGGL(k_pcg_beta, dim3(1), dim3(64), 0, c->stream, a, 1);
    auto iteration = [&]() {
        hipLaunchKernelGGL(k_cg_ap, dim3(kCgBlocks), dim3(kBlock), 0, c->stream, a);
        hipLaunchKernelGGL(k_cg_update, dim3(kCgBlocks), dim3(kBlock), 0, c->stream, a);
        hipLaunchKernelGGL(k_cg_check, dim3(1), dim3(64), 0, c->stream, a);
        vcycle(c, 0, c->r, c->w.mxa[0], c->w.z);
        hipLaunchKernelGGL(k_pcg_rz, dim3(kCgBlocks), dim3(kBlock), 0, c->stream, a, 0);
        hipLaunchKernelGGL(k_pcg_beta, dim3(1), dim3(64), 0, c->stream, a, 0);
        hipLaunchKernelGGL(k_cg_p, dim3(kCgBlocks), dim3(kBlock), 0, c->stream, a);
    };
    // The step solve replays pairs of iterations from a graph captured on a
    // stream of its own (the kernels read the iteration state from the
    // device and return at once after convergence, so every pair is the same
    // launch sequence); the set-up solve launches them directly.
    const bool use_graph = phi == c->buf.phi && with_charge;
    if (use_graph && !c->pcg_exec) {
        bool ok = true;
        if (!c->cap_stream) ok = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) == hipSuccess;
        hipStream_t keep = c->stream;
        if (ok) ok = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            c->stream = c->cap_stream;
            iteration();
            iteration();
            c->stream = keep;
            hipGraph_t gr = nullptr;
            ok = hipStreamEndCapture(c->cap_stream, &gr) == hipSuccess && gr;
            if (ok) ok = hipGraphInstantiate(&c->pcg_exec, gr, nullptr, nullptr, 0) == hipSuccess;
            if (ok) c->pcg_graph = gr;
            else if (gr) (void)hipGraphDestroy(gr);
        }
        if (!ok) {
            c->stream = keep;
            (void)hipGetLastError();
            return fail(c, PIC_E_HIP, "capture of the solver iterations failed");
        }
    }
    State h{};
    int chunk = c->last_iters > 2 ? c->last_iters : 2;
    for (;;) {
        if (use_graph) {
            for (int k = 0; k < chunk; k += 2)
                if (hipGraphLaunch(c->pcg_exec, c->stream) != hipSuccess)
                    return fail(c, PIC_E_HIP, "graph launch failed");
        } else {
            for (int k = 0; k < 8; ++k) iteration();
        }
        chunk = 2;
        pic_status s = hip_ok(c, hipGetLastError(), "solve");
        if (s == PIC_OK)
            s = hip_ok(c, hipMemcpyAsync(&h, c->st, sizeof(State), hipMemcpyDeviceToHost, c->stream), "copy");
        if (s == PIC_OK) s = hip_ok(c, hipStreamSynchronize(c->stream), "sync");
        if (s != PIC_OK) return s;
        if (h.done) break;
    }
    *iters = h.it;
    bool conv = h.rr <= h.rtol * h.rtol * h.bb || h.bb == 0.0;
    if (!conv) return fail(c, PIC_E_NOT_CONVERGED, "the axisymmetric solve did not converge");
    return PIC_OK;
}

pic_status field(pic_rz_ctx* c) {
    const int64_t nn = (int64_t)c->g.nr * c->g.nz;
    hipLaunchKernelGGL(k_field, dim3(grid_of(nn)), dim3(kBlock), 0, c->stream, c->g, c->buf.phi, c->cfg.h,
                       c->buf.field);
    return hip_ok(c, hipGetLastError(), "field");
}

CollArgs coll_args(pic_rz_ctx* c, uint32_t step) {
    CollArgs a{};
    a.g = c->g;
    a.nc = (int64_t)(c->g.nr - 1) * (c->g.nz - 1);
    int64_t off = 0;
    for (int s = 0; s < 3; ++s) {
        a.r[s] = c->buf.r[s];
        a.z[s] = c->buf.z[s];
        a.vr[s] = c->buf.vr[s];
        a.vt[s] = c->buf.vt[s];
        a.vz[s] = c->buf.vz[s];
        a.id[s] = c->buf.id[s];
        a.cap[s] = c->buf.cap[s];
        a.off[s] = off;
        off += c->buf.cap[s];
    }
    a.st = c->st;
    a.cnt = c->w.ccnt;
    a.cpos = c->w.cpos;
    a.crank = c->w.crank;
    a.start = c->w.start;
    a.seg = c->w.seg;
    a.segid = c->w.segid;
    a.sorted = c->w.sorted;
    a.big = c->w.big;
    a.cellof = c->w.cellof;
    a.used = c->w.used;
    a.pflag = c->w.pflag;
    a.ve = c->w.ve;
    a.iflag = c->w.iflag;
    a.vei = c->w.vei;
    a.charge = c->cfg.cu2 ? c->buf.charge : nullptr;
    a.pkey = c->w.pkey;
    a.pslot = c->w.pslot;
    a.pci = c->w.pci;
    a.pce = c->w.pce;
    a.ppi = c->w.ppi;
    a.ppe = c->w.ppe;
    a.pcap = c->buf.cap[1] + c->buf.cap[2];
    a.cu2 = c->cfg.cu2;
    a.xi2 = c->cfg.xi2;
    a.E = c->buf.field;
    a.xs = c->buf.xs;
    a.xs_n = c->cfg.xs_n;
    a.xs_emin = c->cfg.xs_emin;
    a.xs_lnr = std::log(c->cfg.xs_emax / c->cfg.xs_emin);
    for (int k = 0; k < 3; ++k) a.sig_max[k] = c->sig_max[k];
    a.h = c->cfg.h;
    a.dt = c->cfg.dt;
    a.m_ion = c->cfg.m_ion;
    a.xi = c->cfg.xi;
    a.seed = c->cfg.seed;
    a.step = step;
    // Eq. dfi: w(E) = adk_c (20.5 xi^1.5 / E)^(2 n - 1) exp(-6.83 xi^1.5 / E) per fs
    const double n = 3.69 / std::sqrt(c->cfg.xi);
    a.adk_c = 1.52 * std::pow(4.0, n) * c->cfg.xi / (n * std::tgamma(2.0 * n));
    a.adk_e = 2.0 * n - 1.0;
    a.x32 = std::pow(c->cfg.xi, 1.5);
    a.dt_fs = c->cfg.dt * 1e15;
    a.ebsi = 1.5 * a.x32;
    // w dt grows with E below 6.83 xi^1.5 / (2 n - 1) (about 89 GV/m for Cu, above
    // the BSI cut): the field where it reaches 2^-60, by bisection in log space
    a.e_min = 0.0;
    const double emax = std::min(a.ebsi, 6.83 * a.x32 / a.adk_e);
    auto lw = [&](double E) {
        return std::log(a.adk_c * a.dt_fs) + a.adk_e * std::log(20.5 * a.x32 / E) - 6.83 * a.x32 / E;
    };
    const double target = -60.0 * std::log(2.0);
    if (lw(emax) > target) {
        double lo = 1e-6 * emax, hi = emax;
        if (lw(lo) < target) {
            for (int k = 0; k < 200; ++k) {
                const double mid = 0.5 * (lo + hi);
                (lw(mid) < target ? lo : hi) = mid;
            }
            a.e_min = lo;
        }
    }
    return a;
}

// exclusive prefix of m counts into out, the total into st->total; with
// mdev, of the first min(m, *mdev) counts (a length only the device knows:
// the blocks of a grid bounded by m take the chunks in turn)
void scan_u32(pic_rz_ctx* c, const uint32_t* in, uint32_t* out, int64_t m,
              const unsigned long long* mdev = nullptr) {
    if (m <= 4 * (int64_t)kScanChunk) {
        hipLaunchKernelGGL(k_scan<uint32_t>, dim3(1), dim3(kScanBlock), 0, c->stream, in, out, m, c->st, mdev, 1);
        return;
    }
    const int64_t nb = (m + kScanChunk - 1) / kScanChunk;
    const unsigned G = (unsigned)(mdev ? std::min<int64_t>(nb, 256) : nb);
    hipLaunchKernelGGL(k_scan_sums, dim3(G), dim3(kScanBlock), 0, c->stream, in, m, c->w.ssum, mdev);
    hipLaunchKernelGGL(k_scan<uint32_t>, dim3(1), dim3(kScanBlock), 0, c->stream, (const uint32_t*)c->w.ssum,
                       c->w.spre, nb, c->st, mdev, kScanChunk);
    hipLaunchKernelGGL(k_scan_apply, dim3(G), dim3(kScanBlock), 0, c->stream, in, out, m,
                       (const uint32_t*)c->w.spre, mdev);
}

// grouping by (species, cell), ascending id within a cell
void group(pic_rz_ctx* c, const CollArgs& a) {
    const int64_t ncap = c->buf.cap[0] + c->buf.cap[1] + c->buf.cap[2];
    hipLaunchKernelGGL(k_zero_u32, dim3(grid_of(3 * a.nc)), dim3(kBlock), 0, c->stream, a.cnt, 3 * a.nc, c->st);
    for (int s = 0; s < 3; ++s)
        if (c->buf.cap[s] > 0)
            hipLaunchKernelGGL(k_cells, dim3(grid_of(c->buf.cap[s])), dim3(kBlock), 0, c->stream, a, s);
    scan_u32(c, a.cnt, a.start, 3 * a.nc);
    for (int s = 0; s < 3; ++s)
        if (c->buf.cap[s] > 0)
            hipLaunchKernelGGL(k_place, dim3(grid_of(c->buf.cap[s])), dim3(kBlock), 0, c->stream, a, s);
    hipLaunchKernelGGL(k_rank, dim3(grid_of(ncap)), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL(k_sort_big, dim3(kBigBlocks), dim3(kBlock), 0, c->stream, a);
}

// every species in the grouping's order (cell, then id), freed slots dropped
void reorder(pic_rz_ctx* c, const CollArgs& a) {
    for (int s = 0; s < 3; ++s) {
        if (c->buf.cap[s] == 0) continue;
        ReorderArgs r;
        r.r = c->buf.r[s];
        r.z = c->buf.z[s];
        r.vr = c->buf.vr[s];
        r.vt = c->buf.vt[s];
        r.vz = c->buf.vz[s];
        r.id = c->buf.id[s];
        r.charge = (s == 1 && c->cfg.cu2) ? c->buf.charge : nullptr;
        r.tr = c->w.tr;
        r.tz = c->w.tz;
        r.tvr = c->w.tvr;
        r.tvt = c->w.tvt;
        r.tvz = c->w.tvz;
        r.tid = c->w.tid;
        r.tcharge = c->w.tcharge;
        r.sorted = a.sorted;
        r.start = a.start;
        r.first = s * a.nc;
        r.next = s < 2 ? (s + 1) * a.nc : -1;
        r.st = c->st;
        const unsigned G = grid_of(c->buf.cap[s]);
        hipLaunchKernelGGL(k_reorder_gather, dim3(G), dim3(kBlock), 0, c->stream, r);
        hipLaunchKernelGGL(k_reorder_back, dim3(G), dim3(kBlock), 0, c->stream, r, s);
    }
}

// (e, Cu) pairs, (Cu+, Cu) pairs, (e, Cu+) pairs with Cu2+, field
// ionization, then the products; every sort_every steps the particles are
// reordered by cell first (and grouped again)
void collide(pic_rz_ctx* c, uint32_t step) {
    CollArgs a = coll_args(c, step);
    group(c, a);
    if (c->cfg.sort_every > 0 && step % (uint32_t)c->cfg.sort_every == 0) {
        reorder(c, a);
        group(c, a);
    }
    if (c->buf.cap[0] > 0)
        hipLaunchKernelGGL(k_pair, dim3(grid_of(c->buf.cap[0])), dim3(kBlock), 0, c->stream, a, 1);
    if (c->buf.cap[1] > 0)
        hipLaunchKernelGGL(k_pair, dim3(grid_of(c->buf.cap[1])), dim3(kBlock), 0, c->stream, a, 2);
    if (c->cfg.cu2 && c->buf.cap[0] > 0 && c->buf.cap[1] > 0)
        hipLaunchKernelGGL(k_pair, dim3(grid_of(c->buf.cap[0])), dim3(kBlock), 0, c->stream, a, 3);
    if (c->buf.cap[2] > 0) hipLaunchKernelGGL(k_fi, dim3(grid_of(c->buf.cap[2])), dim3(kBlock), 0, c->stream, a);
    if (a.pcap == 0) return;
    hipLaunchKernelGGL(k_prod_list, dim3(grid_of(a.pcap)), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL(k_prod_sort, dim3(1), dim3(1024), 0, c->stream, a);
    // the kernels after the sort cover the list's entries only (its length
    // on the device), with grids bounded by the longest list
    const unsigned Gp = std::min(grid_of(a.pcap), 1024u);
    const unsigned long long* np = &c->st->nprod;
    hipLaunchKernelGGL(k_prod_counts, dim3(Gp), dim3(kBlock), 0, c->stream, a);
    scan_u32(c, a.pci, a.ppi, a.pcap, np);
    scan_u32(c, a.pce, a.ppe, a.pcap, np);
    hipLaunchKernelGGL(k_prod_commit, dim3(1), dim3(64), 0, c->stream, a);
    hipLaunchKernelGGL(k_prod_place, dim3(Gp), dim3(kBlock), 0, c->stream, a);
}

// Fowler-Nordheim emission from the rings of the tip
void emit(pic_rz_ctx* c, uint32_t step) {
    EmitArgs a{};
    a.g = c->g;
    a.phi = c->buf.phi;
    a.rings = c->cfg.fn_rings;
    a.npatch = patches(&c->cfg);
    a.h = c->cfg.h;
    a.dt = c->cfg.dt;
    a.phi_w = c->cfg.phi_w;
    a.phi_w15 = std::pow(c->cfg.phi_w, 1.5);
    a.fn_a = kQe * kQe / (8.0 * kPi * pic::kHpl);
    a.fn_b = (8.0 * kPi / 3.0) * std::sqrt(2.0 * kMe) / (kQe * pic::kHpl) * std::pow(kQe, 1.5);
    a.fn_cs2 = kQe / (4.0 * kPi * kEps0);
    a.seed = c->cfg.seed;
    a.step = step;
    a.cap0 = c->buf.cap[0];
    a.cnt = c->w.pcnt;
    a.offs = c->w.poff;
    a.r = c->buf.r[0];
    a.z = c->buf.z[0];
    a.vr = c->buf.vr[0];
    a.vt = c->buf.vt[0];
    a.vz = c->buf.vz[0];
    a.id = c->buf.id[0];
    a.st = c->st;
    if (a.npatch == 0) return;
    hipLaunchKernelGGL(k_emit_count, dim3(grid_of(a.npatch)), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL(k_scan<uint64_t>, dim3(1), dim3(kScanBlock), 0, c->stream, (const uint32_t*)a.cnt, a.offs,
                       a.npatch, c->st);
    hipLaunchKernelGGL(k_emit_commit, dim3(1), dim3(64), 0, c->stream, c->st, c->buf.cap[0]);
    hipLaunchKernelGGL(k_emit_place, dim3((unsigned)a.npatch), dim3(kBlock), 0, c->stream, a);
}

}  // namespace

extern "C" {

pic_status pic_rz_scratch_size(const pic_rz_config* cfg, const int64_t cap[3], size_t* bytes) {
    if (check(cfg) || !cap || !bytes || !caps_ok(cap)) return PIC_E_INVALID_ARG;
    *bytes = layout(cfg, cap, nullptr, nullptr);
    return PIC_OK;
}

pic_status pic_rz_init(const pic_rz_config* cfg, const pic_rz_buffers* bufs, void* hip_stream, pic_rz_ctx** out) {
    if (!out) return PIC_E_INVALID_ARG;
    *out = nullptr;
    if (check(cfg) || !bufs) return PIC_E_INVALID_ARG;
    if (!bufs->phi || !bufs->phi1 || !bufs->rho || !bufs->field || !bufs->node_type || !bufs->scratch)
        return PIC_E_INVALID_ARG;
    if (!caps_ok(bufs->cap) || bufs->scratch_bytes < layout(cfg, bufs->cap, nullptr, nullptr))
        return PIC_E_INVALID_ARG;
    if (cfg->xs_n > 0 && !bufs->xs) return PIC_E_INVALID_ARG;
    if (cfg->cu2 && bufs->cap[1] > 0 && !bufs->charge) return PIC_E_INVALID_ARG;
    for (int s = 0; s < 3; ++s) {
        if (bufs->n[s] < 0 || bufs->n[s] > bufs->cap[s]) return PIC_E_INVALID_ARG;
        if (bufs->cap[s] > 0 && (!bufs->r[s] || !bufs->z[s] || !bufs->vr[s] || !bufs->vt[s] || !bufs->vz[s] ||
                                 !bufs->id[s]))
            return PIC_E_INVALID_ARG;
    }
    pic_rz_ctx* c = new pic_rz_ctx();
    c->cfg = *cfg;
    c->buf = *bufs;
    c->stream = (hipStream_t)hip_stream;
    c->g.nr = cfg->nr;
    c->g.nz = cfg->nz;
    c->g.R = cfg->tip_r / cfg->h;
    c->g.H = cfg->tip_h / cfg->h;
    // 256-byte alignment of the work memory
    char* base = (char*)(((uintptr_t)bufs->scratch + 255) & ~(uintptr_t)255);
    layout(cfg, bufs->cap, base, &c->w);
    c->mg = mg_dims(cfg->nr, cfg->nz);
    if (cfg->xs_n > 0) {
        // an interpolated value exceeds the largest node at most by rounding
        const int ntab = cfg->cu2 ? 5 : 3, n = cfg->xs_n;
        std::vector<double> t((size_t)ntab * n);
        if (hipMemcpy(t.data(), bufs->xs, t.size() * 8, hipMemcpyDeviceToHost) != hipSuccess) {
            delete c;
            return PIC_E_HIP;
        }
        for (int k = 0; k < n; ++k) {
            c->sig_max[0] = std::max(c->sig_max[0], t[k] + t[n + k] + (cfg->cu2 ? t[3 * n + k] : 0.0));
            c->sig_max[1] = std::max(c->sig_max[1], t[2 * n + k]);
            if (cfg->cu2) c->sig_max[2] = std::max(c->sig_max[2], t[4 * n + k]);
        }
        for (int k = 0; k < 3; ++k) c->sig_max[k] *= 1.0 + 1e-12;
    }
    c->st = c->w.st;
    c->r = c->w.r;
    c->p = c->w.p;
    c->q = c->w.q;
    c->part = c->w.part;
    c->cnt = c->w.cnt;
    const int64_t nn = (int64_t)cfg->nr * cfg->nz;
    State h0{};
    for (int s = 0; s < 3; ++s) h0.n[s] = (unsigned long long)bufs->n[s];
    pic_status s = hip_ok(c, hipMemcpyAsync(c->st, &h0, sizeof(State), hipMemcpyHostToDevice, c->stream), "copy");
    for (int sp = 0; sp < 3 && s == PIC_OK; ++sp)
        if (bufs->n[sp] > 0)
            hipLaunchKernelGGL(k_check_ids, dim3(std::min<unsigned>(1024u, grid_of(bufs->n[sp]))), dim3(kBlock), 0,
                               c->stream, bufs->id[sp], bufs->n[sp], c->st);
    if (s == PIC_OK && cfg->cu2 && bufs->n[1] > 0)
        hipLaunchKernelGGL(k_check_charge, dim3(grid_of(bufs->n[1])), dim3(kBlock), 0, c->stream,
                           (const uint8_t*)bufs->charge, bufs->n[1], c->st);
    if (s == PIC_OK) {
        State h1{};
        s = hip_ok(c, hipMemcpyAsync(&h1, c->st, sizeof(State), hipMemcpyDeviceToHost, c->stream), "copy");
        if (s == PIC_OK) s = hip_ok(c, hipStreamSynchronize(c->stream), "sync");
        if (s == PIC_OK && h1.skip) {
            delete c;
            return PIC_E_INVALID_ARG;
        }
        if (s == PIC_OK) {
            // every species' ids continue from the largest of all
            State h2 = h1;
            h2.skip = 0;
            s = hip_ok(c, hipMemcpyAsync(c->st, &h2, sizeof(State), hipMemcpyHostToDevice, c->stream), "copy");
            if (s == PIC_OK) s = hip_ok(c, hipStreamSynchronize(c->stream), "sync");
        }
    }
    if (s == PIC_OK) {
        hipLaunchKernelGGL(k_types, dim3(grid_of(nn)), dim3(kBlock), 0, c->stream, c->g, bufs->node_type);
        s = hip_ok(c, hipMemsetAsync(bufs->phi1, 0, nn * 8, c->stream), "zero");
        // the multigrid levels: coarse node types, held entries of every
        // level array at zero (they are never written)
        for (int l = 0; l < c->mg.levels && s == PIC_OK; ++l) {
            const int64_t m = (int64_t)c->mg.nr[l] * c->mg.nz[l];
            if (l > 0) {
                hipLaunchKernelGGL(k_mg_types, dim3(grid_of(m)), dim3(kBlock), 0, c->stream, level(c, l - 1),
                                   c->mg.nr[l], c->mg.nz[l], c->mg.sr[l - 1], c->mg.sz[l - 1], c->w.mtype[l]);
                s = hip_ok(c, hipMemsetAsync(c->w.mb[l], 0, m * 8, c->stream), "zero");
            }
            if (s == PIC_OK) s = hip_ok(c, hipMemsetAsync(c->w.mxa[l], 0, m * 8, c->stream), "zero");
            if (s == PIC_OK) s = hip_ok(c, hipMemsetAsync(c->w.mxb[l], 0, m * 8, c->stream), "zero");
        }
        if (s == PIC_OK) s = hip_ok(c, hipMemsetAsync(c->r, 0, nn * 8, c->stream), "zero");
        if (s == PIC_OK) s = hip_ok(c, hipMemsetAsync(c->p, 0, nn * 8, c->stream), "zero");
        if (s == PIC_OK) s = mg_inverse(c);
    }
    int it = 0;
    if (s == PIC_OK) s = cg(c, bufs->phi1, 1.0, false, cfg->laplace_rtol, 1000000, &it);
    if (s == PIC_OK) {
        // F1 = phi1(0, H + 1) / h: the node on the axis one spacing above the apex
        const int kz = (int)std::floor(c->g.H + 1.0);
        const double fz = c->g.H + 1.0 - kz;
        double v[2] = {0.0, 0.0};
        s = hip_ok(c, hipMemcpyAsync(v, bufs->phi1 + (int64_t)kz * cfg->nr, 8, hipMemcpyDeviceToHost, c->stream),
                   "copy");
        if (s == PIC_OK)
            s = hip_ok(c, hipMemcpyAsync(v + 1, bufs->phi1 + (int64_t)(kz + 1) * cfg->nr, 8, hipMemcpyDeviceToHost,
                                         c->stream), "copy");
        if (s == PIC_OK) s = hip_ok(c, hipStreamSynchronize(c->stream), "sync");
        c->F1 = ((1.0 - fz) * v[0] + fz * v[1]) / cfg->h;
        c->V0 = cfg->apex_field / c->F1;
    }
    if (s == PIC_OK) {
        hipLaunchKernelGGL(k_scale_copy, dim3(grid_of(nn)), dim3(kBlock), 0, c->stream, bufs->phi, bufs->phi1, c->V0,
                           nn);
        s = field(c);
    }
    if (s == PIC_OK) s = hip_ok(c, hipMemsetAsync(bufs->rho, 0, nn * 8, c->stream), "zero");
    if (s == PIC_OK) s = hip_ok(c, hipStreamSynchronize(c->stream), "sync");
    if (s != PIC_OK) {
        delete c;
        return s;
    }
    *out = c;
    return PIC_OK;
}

pic_status pic_rz_solve(pic_rz_ctx* c, double rtol, int32_t maxit, pic_solve_info* info) {
    if (!c || !(rtol > 0) || maxit < 1) return PIC_E_INVALID_ARG;
    int it = 0;
    pic_status s = cg(c, c->buf.phi, c->V0, true, rtol, maxit, &it);
    c->last_iters = it;
    if (info) {
        *info = pic_solve_info{};
        info->iterations = it;
        info->converged = s == PIC_OK;
    }
    pic_status sf = field(c);
    return s != PIC_OK ? s : sf;
}

pic_status pic_rz_step(pic_rz_ctx* c, int32_t nsteps, uint32_t flags) {
    if (!c || nsteps < 0) return PIC_E_INVALID_ARG;
    if ((flags & PIC_RZ_COLLIDE) && c->cfg.xs_n == 0) return fail(c, PIC_E_INVALID_ARG, "collisions need tables");
    if ((flags & PIC_RZ_EMIT) && c->cfg.fn_rings == 0) return fail(c, PIC_E_INVALID_ARG, "emission needs rings");
    const double qm[3] = {-kQe / kMe, kQe / c->cfg.m_ion, 0.0};
    const int64_t* cap = c->buf.cap;
    for (int t = 0; t < nsteps; ++t) {
        const uint32_t step = (uint32_t)c->step;
        if (flags & PIC_RZ_EMIT) emit(c, step);
        if (flags & PIC_RZ_PUSH) {
            for (int s = 0; s < 3; ++s) {
                if (cap[s] == 0) continue;
                PushArgs a;
                a.g = c->g;
                a.r = c->buf.r[s];
                a.z = c->buf.z[s];
                a.vr = c->buf.vr[s];
                a.vt = c->buf.vt[s];
                a.vz = c->buf.vz[s];
                a.id = c->buf.id[s];
                a.charge = (s == 1 && c->cfg.cu2) ? c->buf.charge : nullptr;
                a.E = c->buf.field;
                a.kq = qm[s] * c->cfg.dt * c->cfg.dt / c->cfg.h;
                a.sp = s;
                a.st = c->st;
                hipLaunchKernelGGL(k_push, dim3(grid_of(cap[s])), dim3(kBlock), 0, c->stream, a);
            }
        }
        if (flags & PIC_RZ_COLLIDE) collide(c, step);
        if (flags & PIC_RZ_DEPOSIT) {
            const int64_t nn = (int64_t)c->g.nr * c->g.nz;
            hipLaunchKernelGGL(k_zero_rho, dim3(grid_of(nn)), dim3(kBlock), 0, c->stream, c->buf.rho, nn);
            // after this step's grouping (collisions), the grouped particles
            // in grouped order and the ones added since; else every slot
            const int grouped = (flags & PIC_RZ_COLLIDE) ? 1 : 0;
            if (grouped && cap[0] + cap[1] > 0)
                hipLaunchKernelGGL(k_deposit_grouped, dim3(grid_of(cap[0] + cap[1])), dim3(kBlock), 0, c->stream,
                                   coll_args(c, (uint32_t)c->step), c->buf.rho);
            for (int s = 0; s < 2; ++s)
                if (cap[s] > 0)
                    hipLaunchKernelGGL(k_deposit, dim3(grid_of(cap[s])), dim3(kBlock), 0, c->stream, c->g,
                                       c->buf.r[s], c->buf.z[s], c->buf.id[s], (const State*)c->st, s,
                                       (int64_t)(s == 0 ? -1 : 1), c->buf.rho, grouped,
                                       (const uint8_t*)((s == 1 && c->cfg.cu2) ? c->buf.charge : nullptr));
        }
        pic_status st = hip_ok(c, hipGetLastError(), "step");
        if (st != PIC_OK) return st;
        if (flags & PIC_RZ_SOLVE) {
            // the guess: linear extrapolation of the two previous step potentials
            const int64_t nn = (int64_t)c->g.nr * c->g.nz;
            hipLaunchKernelGGL(k_extrap, dim3(grid_of(nn)), dim3(kBlock), 0, c->stream, c->buf.node_type, c->buf.phi,
                               c->w.phi_prev, nn, c->n_prev >= 1 ? 1 : 0);
            c->n_prev = c->n_prev >= 1 ? 2 : 1;
            st = pic_rz_solve(c, c->cfg.step_rtol, c->cfg.maxit, nullptr);
            if (st != PIC_OK) return st;
        } else if (flags & PIC_RZ_FIELD) {
            st = field(c);
            if (st != PIC_OK) return st;
        }
        if (flags & PIC_RZ_ADVANCE) c->step++;
    }
    if (flags & (PIC_RZ_EMIT | PIC_RZ_COLLIDE)) {
        int err = 0;
        pic_status s = hip_ok(c, hipMemcpyAsync(&err, &c->st->error, sizeof(int), hipMemcpyDeviceToHost, c->stream),
                              "copy");
        if (s == PIC_OK) s = hip_ok(c, hipStreamSynchronize(c->stream), "sync");
        if (s != PIC_OK) return s;
        if (err != 0)
            return fail(c, (pic_status)err, err == PIC_E_CAPACITY ? "new particles exceed a species' capacity"
                                                                  : "particle ids exhausted");
    }
    return PIC_OK;
}

pic_status pic_rz_moments(pic_rz_ctx* c, pic_rz_moments_t* out) {
    if (!c || !out) return PIC_E_INVALID_ARG;
    pic_status s = hip_ok(c, hipMemsetAsync(c->cnt, 0, 8 * 8, c->stream), "zero");
    if (s != PIC_OK) return s;
    for (int sp = 0; sp < 3; ++sp)
        if (c->buf.cap[sp] > 0)
            hipLaunchKernelGGL(k_counts, dim3(std::min<unsigned>(1024u, grid_of(c->buf.cap[sp]))), dim3(kBlock), 0,
                               c->stream, c->buf.id[sp], (const State*)c->st, sp, c->cnt + sp,
                               (const uint8_t*)nullptr);
    if (c->cfg.cu2 && c->buf.cap[1] > 0)
        hipLaunchKernelGGL(k_counts, dim3(std::min<unsigned>(1024u, grid_of(c->buf.cap[1]))), dim3(kBlock), 0,
                           c->stream, c->buf.id[1], (const State*)c->st, 1, c->cnt + 4,
                           (const uint8_t*)c->buf.charge);
    const int64_t nn = (int64_t)c->g.nr * c->g.nz;
    hipLaunchKernelGGL(k_qsum, dim3(256), dim3(kBlock), 0, c->stream, c->buf.rho, nn, c->cnt + 3);
    unsigned long long h[8];
    State st{};
    s = hip_ok(c, hipMemcpyAsync(h, c->cnt, sizeof(h), hipMemcpyDeviceToHost, c->stream), "copy");
    if (s == PIC_OK) s = hip_ok(c, hipMemcpyAsync(&st, c->st, sizeof(State), hipMemcpyDeviceToHost, c->stream), "copy");
    if (s == PIC_OK) s = hip_ok(c, hipStreamSynchronize(c->stream), "sync");
    if (s != PIC_OK) return s;
    *out = pic_rz_moments_t{};
    for (int sp = 0; sp < 3; ++sp) {
        out->n_alive[sp] = (int64_t)h[sp];
        for (int k = 0; k < 5; ++k) out->absorbed[sp][k] = (int64_t)st.absorbed[sp][k];
    }
    out->q_total = (int64_t)h[3];
    out->step = c->step;
    out->v0 = c->V0;
    out->apex_field1 = c->F1;
    out->last_cg_iters = c->last_iters;
    out->error = st.error;
    for (int sp = 0; sp < 3; ++sp) out->n_slots[sp] = (int64_t)st.n[sp];
    for (int k = 0; k < 5; ++k) out->events[k] = (int64_t)st.events[k];
    out->injected = (int64_t)st.injected;
    out->next_id = (int64_t)st.next_id;
    out->double_ionizations = (int64_t)st.events[5];
    out->ion_ionizations = (int64_t)st.events[6];
    out->n_cu2 = (int64_t)h[4];
    return PIC_OK;
}

const char* pic_rz_last_error(const pic_rz_ctx* c) { return c ? c->err.c_str() : "no context"; }

void pic_rz_destroy(pic_rz_ctx* c) { delete c; }

}  // extern "C"
