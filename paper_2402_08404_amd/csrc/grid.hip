// grid.hip -- node-grid kernels: node types, node field, prefix scan, and the
// FP64 conjugate-gradient Poisson solver.
//
// Poisson's equation (Sec. 2.1, Eq. poi with boundary conditions bcf1-bcf3) is
// discretized by finite volumes on node control volumes clipped at the lateral
// faces: for a free node i, sum_j f_ij (phi_i - phi_j) = q_i / (eps0 h), with
// f_ij = 1 inside, 1/2 on a lateral face and 1/4 on a lateral edge. The
// operator is applied matrix-free from the node types.
#include <algorithm>

#include "pic_internal.hpp"

namespace pic {

__global__ void k_node_types(Grid g, uint8_t* type) {
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.nn) return;
    int i = (int)(n % g.nx);
    int j = (int)((n / g.nx) % g.ny);
    int k = (int)(n / ((int64_t)g.nx * g.ny));
    uint8_t t = 0;
    if (k == 0) t = 1;
    else if (k == g.nz - 1) t = 2;
    else if (inside_tip(g, (double)i, (double)j, (double)k)) t = 1;
    type[n] = t;
}

hipError_t launch_node_types(pic_ctx* c) {
    int64_t G = (c->g.nn + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_node_types, dim3((unsigned)G), dim3(kBlock), 0, c->stream, c->g, c->buf.node_type);
    return hipGetLastError();
}

// Node field E = -grad phi [V/m]: central differences inside, zero normal
// component on the lateral faces (bcf2), one-sided on the two Dirichlet planes.
template <typename T>
__global__ void k_field(Grid g, const double* __restrict__ phi, typename V4<T>::type* __restrict__ E) {
    int64_t G = gridDim.x;
    int64_t n = xcd_block(blockIdx.x, G) * blockDim.x + threadIdx.x;
    if (n >= g.nn) return;
    int i = (int)(n % g.nx);
    int j = (int)((n / g.nx) % g.ny);
    int k = (int)(n / ((int64_t)g.nx * g.ny));
    int64_t pl = (int64_t)g.nx * g.ny;
    double ex = 0.0, ey = 0.0, ez;
    if (i > 0 && i < g.nx - 1) ex = -(phi[n + 1] - phi[n - 1]) / (2.0 * g.h);
    if (j > 0 && j < g.ny - 1) ey = -(phi[n + g.nx] - phi[n - g.nx]) / (2.0 * g.h);
    if (k == 0) ez = -(phi[n + pl] - phi[n]) / g.h;
    else if (k == g.nz - 1) ez = -(phi[n] - phi[n - pl]) / g.h;
    else ez = -(phi[n + pl] - phi[n - pl]) / (2.0 * g.h);
    typename V4<T>::type v;
    v.x = (T)ex;
    v.y = (T)ey;
    v.z = (T)ez;
    v.w = (T)0;
    E[n] = v;
}

hipError_t launch_field(pic_ctx* c, const double* phi, void* field) {
    int64_t G = (c->g.nn + kBlock - 1) / kBlock;
    if (c->cfg.precision == PIC_F32)
        hipLaunchKernelGGL(k_field<float>, dim3((unsigned)G), dim3(kBlock), 0, c->stream, c->g, phi,
                           (float4*)field);
    else
        hipLaunchKernelGGL(k_field<double>, dim3((unsigned)G), dim3(kBlock), 0, c->stream, c->g, phi,
                           (double4*)field);
    return hipGetLastError();
}

__global__ void k_zero(uint4* p, int64_t n16, uint8_t* tail, int64_t ntail) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t s = (int64_t)gridDim.x * blockDim.x;
    for (; i < n16; i += s) p[i] = make_uint4(0, 0, 0, 0);
    if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

// Zero device memory with a kernel (no memset nodes, so the work can be
// captured in a graph).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    int64_t n16 = (int64_t)(bytes / 16);
    int64_t ntail = (int64_t)(bytes % 16);
    int64_t G = (n16 + kBlock - 1) / kBlock;
    if (G > 16384) G = 16384;
    if (G < 1) G = 1;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)G), dim3(kBlock), 0, s, (uint4*)p, n16,
                       (uint8_t*)p + n16 * 16, ntail);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exclusive prefix scan of uint32 (or of popcounts of uint32 words):
// per-tile reduction, scan of the tile sums in one block, per-tile scan.
constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;

template <bool POP>
__device__ inline uint32_t scan_in(const uint32_t* in, int64_t i, int64_t n) {
    if (i >= n) return 0u;
    uint32_t v = in[i];
    return POP ? (uint32_t)__popc(v) : v;
}

__device__ inline int64_t scan_len(int64_t n, const uint32_t* nd) {
    if (!nd) return n;
    int64_t d = (int64_t)*nd;
    return d < n ? d : n;
}

template <bool POP>
__global__ void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n, const uint32_t* nd,
                              uint32_t* __restrict__ bsum) {
    __shared__ uint32_t sh[kBlock / 64];
    n = scan_len(n, nd);
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) s += scan_in<POP>(in, base + k * kBlock + threadIdx.x, n);
    uint32_t t = block_sum(s, sh);
    if (threadIdx.x == 0) bsum[blockIdx.x] = t;
}

// Exclusive scan of the tile sums in one block (any count); writes the total.
__global__ void k_scan_top(uint32_t* bsum, int64_t nb, uint32_t* total) {
    // chunks of kBlock x 8 block sums: each thread scans 8 consecutive
    // values (loaded together: the index is clamped, the value masked), the
    // threads' totals are scanned by wavefront shuffles and the four
    // wavefront totals through LDS
    constexpr int kPer = 8;
    __shared__ uint32_t wsum[kBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += (int64_t)kBlock * kPer) {
        const int64_t base = b0 + (int64_t)threadIdx.x * kPer;
        uint32_t v[kPer];
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int64_t idx = base + q < nb ? base + q : nb - 1;
            const uint32_t x = bsum[idx];
            v[q] = base + q < nb ? x : 0u;
        }
        uint32_t s = 0;
#pragma unroll
        for (int q = 0; q < kPer; ++q) s += v[q];
        uint32_t x = s;  // inclusive scan of the threads' totals in the wavefront
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        uint32_t wpre = 0, tot = 0;
#pragma unroll
        for (int q = 0; q < kBlock / 64; ++q) {
            const uint32_t t = wsum[q];
            wpre += q < w ? t : 0u;
            tot += t;
        }
        uint32_t run = carry + wpre + x - s;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            if (base + q < nb) bsum[base + q] = run;
            run += v[q];
        }
        carry += tot;
        __syncthreads();  // wsum is rewritten by the next chunk
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

template <bool POP>
__global__ void k_scan_down(uint32_t* __restrict__ in, int64_t n, const uint32_t* nd,
                            const uint32_t* __restrict__ bsum, uint32_t* __restrict__ out, int zero_in) {
    __shared__ uint32_t tile[kScanTile];
    __shared__ uint32_t sh[kBlock];
    n = scan_len(n, nd);
    if ((int64_t)blockIdx.x * kScanTile >= n) return;
    int64_t base = (int64_t)blockIdx.x * kScanTile;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k * kBlock + threadIdx.x;
        tile[k * kBlock + threadIdx.x] = scan_in<POP>(in, i, n);
        if (zero_in && i < n) in[i] = 0u;
    }
    __syncthreads();
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) s += tile[threadIdx.x * kScanItems + k];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
        uint32_t add = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0u;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t run = bsum[blockIdx.x] + sh[threadIdx.x] - s;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        uint32_t v = tile[threadIdx.x * kScanItems + k];
        tile[threadIdx.x * kScanItems + k] = run;
        run += v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k * kBlock + threadIdx.x;
        if (i < n) out[i] = tile[k * kBlock + threadIdx.x];
    }
}

// out[i] = sum of in[0..i) for i < n and *total = sum of all, where n is
// n_max or, when nd is given, min(n_max, *nd) read on the device. With
// zero_in the input is cleared in the same pass (in and out may not alias).
hipError_t scan_u32(pic_ctx* c, const uint32_t* in, uint32_t* out, int64_t n_max, const uint32_t* nd,
                    uint32_t* total, bool zero_in, bool popcount) {
    int64_t nb = (n_max + kScanTile - 1) / kScanTile;
    if (nb < 1) nb = 1;
    if (nb > c->scan_blocks_n) return hipErrorInvalidValue;
    if (popcount)
        hipLaunchKernelGGL(k_scan_reduce<true>, dim3((unsigned)nb), dim3(kBlock), 0, c->stream, in, n_max, nd,
                           c->scan_blocks);
    else
        hipLaunchKernelGGL(k_scan_reduce<false>, dim3((unsigned)nb), dim3(kBlock), 0, c->stream, in, n_max, nd,
                           c->scan_blocks);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, c->stream, c->scan_blocks, nb, total);
    if (popcount)
        hipLaunchKernelGGL(k_scan_down<true>, dim3((unsigned)nb), dim3(kBlock), 0, c->stream, (uint32_t*)in, n_max,
                           nd, c->scan_blocks, out, zero_in ? 1 : 0);
    else
        hipLaunchKernelGGL(k_scan_down<false>, dim3((unsigned)nb), dim3(kBlock), 0, c->stream, (uint32_t*)in,
                           n_max, nd, c->scan_blocks, out, zero_in ? 1 : 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Conjugate gradients. Two kernels per iteration over a fixed grid of
// kCgBlocks blocks, each block owning a contiguous chunk of nodes (chunks of
// one XCD are adjacent, so stencil neighbours stay in that XCD's L2). A
// reduction is finished by the next kernel: every block sums the previous
// kernel's per-block partials in the same fixed order (deterministic, and no
// device-wide fence, which on this GPU would write back the whole L2). The
// scalars live on the device; kernels return at once when the solve is done,
// so the host enqueues iterations in chunks and tests convergence per chunk.

constexpr int kCgBlocks = 1024;

struct CgArgs {
    Grid g;
    const uint8_t* type;
    double* x;
    double* r;
    const double* p_old;
    double* p_new;
    double* q;
    const int64_t* rho;
    double qscale;   // 2^-40 e / (eps0 h)
    double V0;
    const double* V0_dev;   // when set, the anode value (the circuit's gap voltage) is read here
    DevState* s;
    double* part_pq;  // kCgBlocks partials of p.q
    double* part_rr;  // kCgBlocks partials of r.r
    double* part_bb;  // kCgBlocks partials of b.b
    int64_t chunk;    // nodes per block (multiple of the block size)
};

__device__ inline double half_at_edge(int i, int n) { return (i == 0 || i == n - 1) ? 0.5 : 1.0; }

__device__ inline void node_ijk(const Grid& g, int64_t n, int& i, int& j, int& k) {
    i = (int)(n % g.nx);
    j = (int)((n / g.nx) % g.ny);
    k = (int)(n / ((int64_t)g.nx * g.ny));
}

// Sum of the kCgBlocks partials of the previous kernel, in a fixed order.
__device__ inline double sum_partials(const double* part) { return sum_partials_n(part, kCgBlocks); }

__device__ inline void write_partial(double v, double* part) {
    __shared__ double sh[kBlock / 64];
    double t = block_sum(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Dirichlet values into phi, optional zero guess.
__global__ void k_cg_init(CgArgs a, int zero_guess) {
    const Grid& g = a.g;
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.nn) return;
    uint8_t t = a.type[n];
    if (t != 0) {
        a.x[n] = (t == 2) ? (a.V0_dev ? *a.V0_dev : a.V0) : 0.0;
        a.r[n] = 0.0;
    } else if (zero_guess) {
        a.x[n] = 0.0;
    }
}

// r = q/(eps0 h) - L(phi) with the Dirichlet values in phi, partials of r.r
// and of b.b with b = q/(eps0 h) + Dirichlet lifts; p_old cleared. Blocks of
// kResidBlock threads over the same kCgBlocks chunks as the CG kernels (so
// the partial counts match); neighbour loads are unconditional (read at the
// node itself with weight zero at the grid faces), so a node's loads are in
// flight together.
constexpr int kResidBlock = 1024;

__global__ __launch_bounds__(kResidBlock) void k_cg_resid(CgArgs a) {
    const Grid& g = a.g;
    int64_t b0 = xcd_block(blockIdx.x, gridDim.x) * a.chunk;
    int64_t b1 = b0 + a.chunk < g.nn ? b0 + a.chunk : g.nn;
    const int64_t pl = (int64_t)g.nx * g.ny;
    double bb = 0.0, rr = 0.0;
    NodeWalk wk(b0 + threadIdx.x, blockDim.x, g.nx, g.ny);
    for (int64_t n = b0 + threadIdx.x; n < b1; n += blockDim.x, wk.advance()) {
        ((double*)a.p_old)[n] = 0.0;
        const int i = wk.i, j = wk.j, k = wk.k;
        const double fx = half_at_edge(j, g.ny) * half_at_edge(k, g.nz);
        const double fy = half_at_edge(i, g.nx) * half_at_edge(k, g.nz);
        const double fz = half_at_edge(i, g.nx) * half_at_edge(j, g.ny);
        const bool hs[6] = {i > 0, i < g.nx - 1, j > 0, j < g.ny - 1, k > 0, k < g.nz - 1};
        const int64_t d[6] = {-1, 1, -(int64_t)g.nx, (int64_t)g.nx, -pl, pl};
        const double f[6] = {fx, fx, fy, fy, fz, fz};
        const double xi = a.x[n];
        const bool fr = a.type[n] == 0;
        const double qv = (double)a.rho[n] * a.qscale;
        double xj[6];
        uint8_t tj[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const int64_t m = hs[q] ? n + d[q] : n;
            xj[q] = a.x[m];
            tj[q] = a.type[m];
        }
        double lx = 0.0, bv = qv;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const double w = hs[q] ? f[q] : 0.0;
            lx += w * (xi - xj[q]);
            bv += (tj[q] != 0 ? w : 0.0) * xj[q];
        }
        const double rv = qv - lx;
        if (fr) {
            a.r[n] = rv;
            bb += bv * bv;
            rr += rv * rv;
        }
    }
    __shared__ double sh[kResidBlock / 64];
    const double tb = block_sum(bb, sh);
    if (threadIdx.x == 0) a.part_bb[blockIdx.x] = tb;
    const double tr = block_sum(rr, sh);
    if (threadIdx.x == 0) a.part_rr[blockIdx.x] = tr;
}

// The same residual as a z-marching kernel (see ZMarch): the values and
// node types of the planes below and above come from registers, the
// in-plane neighbours from L1/L2. At most kCgBlocks blocks; block 0 clears
// the partial slots of the blocks that do not exist, so the consumers sum
// kCgBlocks partials as for k_cg_resid.
__global__ __launch_bounds__(kBlock) void k_cg_resid_z(CgArgs a, int kc) {
    const Grid& g = a.g;
    const ZMarch t = zmarch(g.nx, g.ny, g.nz, kc);
    const int64_t pl = (int64_t)g.nx * g.ny;
    double bb = 0.0, rr = 0.0;
    if (t.col) {
        const int i = t.i, j = t.j;
        const double hx = half_at_edge(i, g.nx), hy = half_at_edge(j, g.ny);
        // neighbours outside the grid are read at the node itself with weight
        // zero, so every load is unconditional
        const int64_t ow = i > 0 ? -1 : 0, oe = i < g.nx - 1 ? 1 : 0;
        const int64_t os = j > 0 ? -(int64_t)g.nx : 0, on = j < g.ny - 1 ? (int64_t)g.nx : 0;
        int64_t n = (int64_t)t.k0 * pl + (int64_t)j * g.nx + i;
        double xm = a.x[t.k0 > 0 ? n - pl : n], xc = a.x[n];
        uint8_t tm = a.type[t.k0 > 0 ? n - pl : n], tc = a.type[n];
        for (int k = t.k0; k < t.k1; ++k, n += pl) {
            const bool up = k + 1 < g.nz;
            const double xp = a.x[up ? n + pl : n];
            const uint8_t tp = a.type[up ? n + pl : n];
            const double xw = a.x[n + ow], xe = a.x[n + oe], xs = a.x[n + os], xn = a.x[n + on];
            const uint8_t tw = a.type[n + ow], te = a.type[n + oe], ts = a.type[n + os], tn = a.type[n + on];
            const double qv = (double)a.rho[n] * a.qscale;
            ((double*)a.p_old)[n] = 0.0;
            const double hz = half_at_edge(k, g.nz);
            const double fx = hy * hz, fy = hx * hz, fz = hx * hy;
            const double xj[6] = {xw, xe, xs, xn, xm, xp};
            const uint8_t tj[6] = {tw, te, ts, tn, tm, tp};
            const double w[6] = {i > 0 ? fx : 0.0, i < g.nx - 1 ? fx : 0.0, j > 0 ? fy : 0.0,
                                 j < g.ny - 1 ? fy : 0.0, k > 0 ? fz : 0.0, up ? fz : 0.0};
            double lx = 0.0, bv = qv;
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                lx += w[q] * (xc - xj[q]);
                bv += (tj[q] != 0 ? w[q] : 0.0) * xj[q];
            }
            const double rv = qv - lx;
            if (tc == 0) {
                a.r[n] = rv;
                bb += bv * bv;
                rr += rv * rv;
            }
            xm = xc;
            xc = xp;
            tm = tc;
            tc = tp;
        }
    }
    __shared__ double sh[kBlock / 64];
    const double tb = block_sum(bb, sh);
    if (threadIdx.x == 0) a.part_bb[blockIdx.x] = tb;
    const double tr = block_sum(rr, sh);
    if (threadIdx.x == 0) a.part_rr[blockIdx.x] = tr;
    if (blockIdx.x == 0)
        for (int b = (int)gridDim.x + (int)threadIdx.x; b < kCgBlocks; b += kBlock) a.part_bb[b] = a.part_rr[b] = 0.0;
}

// Initial residual and its partials: the z-marching kernel where the grid
// fits in kCgBlocks blocks, else k_cg_resid.
static void launch_resid(pic_ctx* c, const CgArgs& a) {
    const Grid& g = a.g;
    const int64_t cols = (int64_t)((g.nx + 63) / 64) * ((g.ny + 3) / 4);
    if (cols <= kCgBlocks) {
        int64_t kc = (g.nz * cols + kCgBlocks - 1) / kCgBlocks;
        while (cols * ((g.nz + kc - 1) / kc) > kCgBlocks) ++kc;
        const unsigned zb = (unsigned)(cols * ((g.nz + kc - 1) / kc));
        hipLaunchKernelGGL(k_cg_resid_z, dim3(zb), dim3(kBlock), 0, c->stream, a, (int)kc);
    } else {
        hipLaunchKernelGGL(k_cg_resid, dim3(kCgBlocks), dim3(kResidBlock), 0, c->stream, a);
    }
}

// Iteration it: finish r.r of the previous iteration (or of the initial
// residual), test convergence, then p_new = r + beta p_old, q = A p_new and
// the partials of p_new . q.
__global__ __launch_bounds__(kBlock) void k_cg_a(CgArgs a, int it) {
    DevState* s = a.s;
    if (s->done) return;
    const Grid& g = a.g;
    double rr = sum_partials(a.part_rr);
    double bb;
    if (it == 0) {
        bb = sum_partials(a.part_bb);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            s->bb = bb;
            s->rr0 = rr;
        }
    } else {
        bb = s->bb;
    }
    bool conv = (bb == 0.0) || (sqrt(rr) <= s->rtol * sqrt(bb)) || (it >= s->maxit);
    double beta = it == 0 ? 0.0 : rr / s->rrbuf[(it - 1) & 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s->rrbuf[it & 1] = rr;
        s->rr = rr;
        s->it = it;
        if (conv) {
            s->done = 1;
            s->zero_solution = (bb == 0.0);
        }
    }
    if (conv) return;
    int64_t b0 = xcd_block(blockIdx.x, gridDim.x) * a.chunk;
    int64_t b1 = b0 + a.chunk < g.nn ? b0 + a.chunk : g.nn;
    int64_t pl = (int64_t)g.nx * g.ny;
    double pq = 0.0;
    NodeWalk wk(b0 + threadIdx.x, blockDim.x, g.nx, g.ny);
    for (int64_t n = b0 + threadIdx.x; n < b1; n += blockDim.x, wk.advance()) {
        if (a.type[n] != 0) {
            a.p_new[n] = 0.0;
            a.q[n] = 0.0;
            continue;
        }
        int i = wk.i, j = wk.j, k = wk.k;
        double fx = half_at_edge(j, g.ny) * half_at_edge(k, g.nz);
        double fy = half_at_edge(i, g.nx) * half_at_edge(k, g.nz);
        double fz = half_at_edge(i, g.nx) * half_at_edge(j, g.ny);
        double pi = a.r[n] + beta * a.p_old[n];
        double acc = 0.0;
        int64_t nb[6] = {n - 1, n + 1, n - g.nx, n + g.nx, n - pl, n + pl};
        bool has[6] = {i > 0, i < g.nx - 1, j > 0, j < g.ny - 1, true, true};
        double f[6] = {fx, fx, fy, fy, fz, fz};
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            if (!has[d]) continue;
            int64_t m = nb[d];
            double pj = a.r[m] + beta * a.p_old[m];  // r and p are zero on fixed nodes
            acc += f[d] * (pi - pj);
        }
        a.p_new[n] = pi;
        a.q[n] = acc;
        pq += pi * acc;
    }
    write_partial(pq, a.part_pq);
}

// Iteration it: alpha = rr / pq, x += alpha p, r -= alpha q, partials of r.r.
__global__ __launch_bounds__(kBlock) void k_cg_b(CgArgs a, int it) {
    DevState* s = a.s;
    if (s->done) return;
    const Grid& g = a.g;
    double pq = sum_partials(a.part_pq);
    double alpha = s->rrbuf[it & 1] / pq;
    int64_t b0 = xcd_block(blockIdx.x, gridDim.x) * a.chunk;
    int64_t b1 = b0 + a.chunk < g.nn ? b0 + a.chunk : g.nn;
    double rr = 0.0;
    // p and q are zero on fixed nodes, so x and r keep their values there
    // and no node type is needed
    for (int64_t n = b0 + threadIdx.x; n < b1; n += blockDim.x) {
        double p = a.p_new[n];
        a.x[n] += alpha * p;
        double r = a.r[n] - alpha * a.q[n];
        a.r[n] = r;
        rr += r * r;
    }
    write_partial(rr, a.part_rr);
    if (blockIdx.x == 0 && threadIdx.x == 0) s->it = it + 1;
}

__global__ void k_cg_zero_free(Grid g, const uint8_t* type, double* x, const DevState* s) {
    if (!s->zero_solution) return;
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n < g.nn && type[n] == 0) x[n] = 0.0;
}

__global__ void k_cg_setup(DevState* s, double rtol, int maxit) {
    s->rtol = rtol;
    s->maxit = maxit;
    s->done = 0;
    s->it = 0;
    s->zero_solution = 0;
}

int cg_solve(pic_ctx* c, double* phi, double V0, const int64_t* rho, int guess, double rtol, int maxit,
             pic_solve_info* info) {
    const Grid& g = c->g;
    int64_t G = (g.nn + kBlock - 1) / kBlock;
    CgArgs a;
    a.g = g;
    a.type = c->buf.node_type;
    a.x = phi;
    a.r = c->cg_r;
    a.p_old = c->cg_p0;
    a.p_new = c->cg_p1;
    a.q = c->cg_q;
    a.rho = rho;
    a.qscale = ldexp(1.0, -40) * kQe / (kEps0 * g.h);
    a.V0 = V0;
    a.V0_dev = (c->circuit && phi == c->buf.phi) ? &c->st->v_gap : nullptr;
    a.s = c->st;
    a.part_pq = c->partials;
    a.part_rr = c->partials + kCgBlocks;
    a.part_bb = c->partials + 2 * kCgBlocks;
    a.chunk = ((g.nn + kCgBlocks - 1) / kCgBlocks + kBlock - 1) / kBlock * kBlock;
    hipLaunchKernelGGL(k_cg_setup, dim3(1), dim3(1), 0, c->stream, c->st, rtol, maxit);
    hipLaunchKernelGGL(k_cg_init, dim3((unsigned)G), dim3(kBlock), 0, c->stream, a, guess == PIC_GUESS_ZERO);
    launch_resid(c, a);
    double* pa = c->cg_p0;
    double* pb = c->cg_p1;
    int chunk = 8;
    int launched = 0;
    while (true) {
        for (int t = 0; t < chunk && launched <= maxit; ++t, ++launched) {
            a.p_old = pa;
            a.p_new = pb;
            bool timed = launched < 256;  // per-kernel timing of the first iterations only
            int ta = timed ? tic(c, PIC_T_CG_A) : -1;
            hipLaunchKernelGGL(k_cg_a, dim3(kCgBlocks), dim3(kBlock), 0, c->stream, a, launched);
            toc(c, ta);
            if (launched == maxit) continue;  // the last launch only finishes r.r and the test
            int tb = timed ? tic(c, PIC_T_CG_B) : -1;
            hipLaunchKernelGGL(k_cg_b, dim3(kCgBlocks), dim3(kBlock), 0, c->stream, a, launched);
            toc(c, tb);
            double* t2 = pa;
            pa = pb;
            pb = t2;
        }
        (void)hipMemcpyAsync(c->host_st, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream);
        if (hipStreamSynchronize(c->stream) != hipSuccess) return -2;
        if (c->host_st->done || launched > maxit) break;
        if (chunk < 64) chunk *= 2;
    }
    hipLaunchKernelGGL(k_cg_zero_free, dim3((unsigned)G), dim3(kBlock), 0, c->stream, g, c->buf.node_type, phi,
                       c->st);
    (void)hipMemcpyAsync(c->host_st, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return -2;
    const DevState* h = c->host_st;
    double bn = sqrt(h->bb);
    info->iterations = h->it;
    info->relres = h->zero_solution ? 0.0 : sqrt(h->rr) / bn;
    info->relres0 = h->zero_solution ? 0.0 : sqrt(h->rr0) / bn;
    info->converged = h->zero_solution || (sqrt(h->rr) <= rtol * bn);
    return 0;
}

// ---------------------------------------------------------------------------
// CG preconditioned by the multigrid V-cycle (z = M r, z in FP32). Per
// iteration: the V-cycle (its first kernel finishes r.r and tests
// convergence, its last writes the partials of r.z), then k_pcg_a (beta from
// r.z, p = z + beta p, q = A p, partials of p.q) and k_pcg_b (alpha, x and r
// update, partials of r.r). The iteration count and the previous r.z live on
// the device, so every iteration launches the same kernels with the same
// arguments. TP is the type of the Krylov vectors x, r, p, q: FP64 for the
// multigrid-preconditioned solver, FP32 for the inner solves of the
// mixed-precision one. Dot products are always accumulated in FP64.

template <typename TP>
struct PcgArgs {
    Grid g;
    const uint8_t* type;
    TP* x;
    TP* r;
    const TP* p_old;
    TP* p_new;
    TP* q;
    DevState* s;
    double* part_pq;
    double* part_rr;
    int64_t chunk;
};

// z-marching: p = z + beta p_old at the node and its six neighbours, q = A p.
template <typename TP>
__global__ __launch_bounds__(kBlock) void k_pcg_a(PcgArgs<TP> a, const float* __restrict__ z, const double* part_rz,
                                                   int n_rz, int kc) {
    DevState* s = a.s;
    if (s->done) return;
    const Grid& g = a.g;
    double rz = sum_partials_n(part_rz, n_rz);
    double beta = s->it == 0 ? 0.0 : rz / s->rz_prev;
    const TP* __restrict__ po = a.p_old;
    auto pv = [&](int64_t m) { return (double)z[m] + beta * (double)po[m]; };  // zero on fixed nodes
    ZMarch t = zmarch(g.nx, g.ny, g.nz, kc);
    double pq = 0.0;
    if (t.col) {
        int i = t.i, j = t.j;
        int64_t pl = (int64_t)g.nx * g.ny;
        int64_t n = (int64_t)t.k0 * pl + (int64_t)j * g.nx + i;
        double hx = half_at_edge(i, g.nx), hy = half_at_edge(j, g.ny), fz = hx * hy;
        // neighbours outside the grid are read at the node itself with a zero
        // weight: every load is unconditional, so a step's loads issue together
        const int64_t ow = i > 0 ? -1 : 0, oe = i < g.nx - 1 ? 1 : 0;
        const int64_t os = j > 0 ? -(int64_t)g.nx : 0, on = j < g.ny - 1 ? (int64_t)g.nx : 0;
        // a free node is never on a z face: fx = hy, fy = hx
        const double ww = i > 0 ? hy : 0.0, we = i < g.nx - 1 ? hy : 0.0;
        const double ws = j > 0 ? hx : 0.0, wn = j < g.ny - 1 ? hx : 0.0;
        double pm = pv(t.k0 > 0 ? n - pl : n);
        if (t.k0 == 0) pm = 0.0;
        double pc = pv(n);
        for (int k = t.k0; k < t.k1; ++k, n += pl) {
            const bool up = k + 1 < g.nz;
            double pp = pv(up ? n + pl : n);
            if (!up) pp = 0.0;
            const double xw = pv(n + ow), xe = pv(n + oe), xs = pv(n + os), xn = pv(n + on);
            const bool fr = a.type[n] == 0;
            double acc = 0.0;
            acc += ww * (pc - xw);
            acc += we * (pc - xe);
            acc += ws * (pc - xs);
            acc += wn * (pc - xn);
            acc += fz * (pc - pm);
            acc += fz * (pc - pp);
            const TP pn = (TP)pc, qn = (TP)(fr ? acc : 0.0);
            pq += (double)pn * (double)qn;
            a.p_new[n] = pn;
            a.q[n] = qn;
            pm = pc;
            pc = pp;
        }
    }
    __shared__ double sh[kBlock / 64];
    double tsum = block_sum(pq, sh);
    if (threadIdx.x == 0) a.part_pq[blockIdx.x] = tsum;
}

// Pair variant of k_pcg_a for FP64 Krylov vectors and an even nx: each lane
// owns two adjacent x nodes (16-byte loads and stores of FP64 pairs), a wave
// covers 128 consecutive x nodes of one row, and the x neighbours of the pair
// come from the adjacent lanes by shuffles (from memory at the ends of the
// 128-node segment). Lanes past the grid edge compute on clamped addresses and
// store nothing, so every lane takes part in the shuffles.
__global__ __launch_bounds__(kBlock) void k_pcg_a2(PcgArgs<double> a, const float* __restrict__ z,
                                                    const double* part_rz, int n_rz, int kc) {
    DevState* s = a.s;
    if (s->done) return;
    const Grid& g = a.g;
    const double rz = sum_partials_n(part_rz, n_rz);
    const double beta = s->it == 0 ? 0.0 : rz / s->rz_prev;
    const double* __restrict__ po = a.p_old;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int ntx = (g.nx + 127) >> 7, nty = (g.ny + 3) >> 2;
    const int64_t b = xcd_block(blockIdx.x, gridDim.x);
    const int bx = (int)(b % ntx);
    const int64_t rr = b / ntx;
    const int by = (int)(rr % nty), bz = (int)(rr / nty);
    const int i0 = bx * 128 + 2 * lane, j = by * 4 + w;
    const int k0 = bz * kc, k1 = k0 + kc < g.nz ? k0 + kc : g.nz;
    const bool col = i0 < g.nx && j < g.ny;
    const int ic = col ? i0 : 0, jc = j < g.ny ? j : g.ny - 1;
    const int64_t pl = (int64_t)g.nx * g.ny;
    int64_t n = (int64_t)k0 * pl + (int64_t)jc * g.nx + ic;
    auto pv2 = [&](int64_t m) {
        const float2 zz = *(const float2*)(z + m);
        const double2 pp = *(const double2*)(po + m);
        return make_double2((double)zz.x + beta * pp.x, (double)zz.y + beta * pp.y);
    };
    auto pv1 = [&](int64_t m) { return (double)z[m] + beta * po[m]; };
    const double hx0 = half_at_edge(ic, g.nx), hx1 = half_at_edge(ic + 1, g.nx), hy = half_at_edge(jc, g.ny);
    const double fz0 = hx0 * hy, fz1 = hx1 * hy;
    const bool hasW = ic > 0, hasE = ic + 2 < g.nx;
    const int64_t os = jc > 0 ? -(int64_t)g.nx : 0, on = jc < g.ny - 1 ? (int64_t)g.nx : 0;
    const double ws0 = jc > 0 ? hx0 : 0.0, ws1 = jc > 0 ? hx1 : 0.0;
    const double wn0 = jc < g.ny - 1 ? hx0 : 0.0, wn1 = jc < g.ny - 1 ? hx1 : 0.0;
    double2 pm = pv2(k0 > 0 ? n - pl : n);
    if (k0 == 0) pm = make_double2(0.0, 0.0);
    double2 pc = pv2(n);
    double pq = 0.0;
    for (int k = k0; k < k1; ++k, n += pl) {
        const bool up = k + 1 < g.nz;
        double2 pp = pv2(up ? n + pl : n);
        if (!up) pp = make_double2(0.0, 0.0);
        const double2 ps = pv2(n + os), pn = pv2(n + on);
        const uint16_t tt = *(const uint16_t*)(a.type + n);
        double left = __shfl_up(pc.y, 1), right = __shfl_down(pc.x, 1);
        if (lane == 0) left = hasW ? pv1(n - 1) : 0.0;
        if (lane == 63) right = hasE ? pv1(n + 2) : 0.0;
        // a free node is never on a z face: fx = hy, fy = hx
        double acc0 = 0.0;
        acc0 += (hasW ? hy : 0.0) * (pc.x - left);
        acc0 += hy * (pc.x - pc.y);
        acc0 += ws0 * (pc.x - ps.x);
        acc0 += wn0 * (pc.x - pn.x);
        acc0 += fz0 * (pc.x - pm.x);
        acc0 += fz0 * (pc.x - pp.x);
        double acc1 = 0.0;
        acc1 += hy * (pc.y - pc.x);
        acc1 += (hasE ? hy : 0.0) * (pc.y - right);
        acc1 += ws1 * (pc.y - ps.y);
        acc1 += wn1 * (pc.y - pn.y);
        acc1 += fz1 * (pc.y - pm.y);
        acc1 += fz1 * (pc.y - pp.y);
        const double q0 = (tt & 0xff) == 0 ? acc0 : 0.0, q1 = (tt >> 8) == 0 ? acc1 : 0.0;
        if (col) {
            pq += pc.x * q0;
            pq += pc.y * q1;
            *(double2*)(a.p_new + n) = pc;
            *(double2*)(a.q + n) = make_double2(q0, q1);
        }
        pm = pc;
        pc = pp;
    }
    __shared__ double sh[kBlock / 64];
    double tsum = block_sum(pq, sh);
    if (threadIdx.x == 0) a.part_pq[blockIdx.x] = tsum;
}

// Grid of k_pcg_a2: 128 x 4 (x, y) tiles, kc planes per block, about
// `target` blocks.
static unsigned pair_grid(int nx, int ny, int nz, int target, int* kc) {
    int64_t cols = (int64_t)((nx + 127) / 128) * ((ny + 3) / 4);
    int64_t k = (nz * cols + target - 1) / target;
    if (k < 1) k = 1;
    while (k < nz && cols * ((nz + k - 1) / k) > kMaxStencilBlocks) ++k;  // partial-sum slots
    *kc = (int)k;
    return (unsigned)(cols * ((nz + k - 1) / k));
}

template <typename TP>
__global__ __launch_bounds__(kBlock) void k_pcg_b(PcgArgs<TP> a, const double* part_rz, int n_rz, int n_pq) {
    DevState* s = a.s;
    if (s->done) return;
    const Grid& g = a.g;
    double rz = sum_partials_n(part_rz, n_rz);
    double pq = sum_partials_n(a.part_pq, n_pq);
    double alpha = rz / pq;
    int64_t b0 = xcd_block(blockIdx.x, gridDim.x) * a.chunk;
    int64_t b1 = b0 + a.chunk < g.nn ? b0 + a.chunk : g.nn;
    double rr = 0.0;
    // p and q are zero on fixed nodes, so x and r keep their values there
    // and no node type is needed
    for (int64_t n = b0 + threadIdx.x; n < b1; n += blockDim.x) {
        double p = a.p_new[n];
        a.x[n] = (TP)((double)a.x[n] + alpha * p);
        double r = (double)a.r[n] - alpha * (double)a.q[n];
        TP rn = (TP)r;
        a.r[n] = rn;
        rr += (double)rn * (double)rn;
    }
    __shared__ double sh[kBlock / 64];
    double tsum = block_sum(rr, sh);
    if (threadIdx.x == 0) a.part_rr[blockIdx.x] = tsum;
    // only this block reads or writes the iteration state in this kernel
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s->rz_prev = rz;
        s->it = s->it + 1;
    }
}

// Partials of the mixed-precision refinement live after the CG ones.
constexpr int kPartPq = 0, kPartRr = 4096, kPartBb = 8192, kPartRz = 12288;

// Run the preconditioned iterations on x, r (type TP; r also the V-cycle's
// right-hand side) after k_cg_setup and the partials of r.r and b.b are in
// place. p0, p1, q: work vectors of type TP. slot selects the captured graph
// (0: FP64 solver, 1: inner FP32 solver). Returns 0, or -2 on a HIP error.
template <typename TP>
static int pcg_iterate(pic_ctx* c, TP* x, TP* r, TP* p0, TP* p1, TP* q, int maxit, int slot) {
    const Grid& g = c->g;
    PcgArgs<TP> a;
    a.g = g;
    a.type = c->buf.node_type;
    a.x = x;
    a.r = r;
    a.q = q;
    a.s = c->st;
    a.part_pq = c->partials + kPartPq;
    a.part_rr = c->partials + kPartRr;
    double* part_bb = c->partials + kPartBb;
    double* part_rz = c->partials + kPartRz;
    a.chunk = ((g.nn + kCgBlocks - 1) / kCgBlocks + kBlock - 1) / kBlock * kBlock;
    int kc = 1;
    // FP64 vectors on a grid of even width take the pair kernel
    const bool pair = sizeof(TP) == 8 && (g.nx % 2) == 0;
    unsigned zb = pair ? pair_grid(g.nx, g.ny, g.nz, stencil_target(c), &kc)
                       : zmarch_grid(g.nx, g.ny, g.nz, stencil_target(c), 1, &kc);
    if (zb > kMaxStencilBlocks) return -3;
    // one iteration: V-cycle, p update and A p, x and r update
    auto iteration = [&](TP* p_old, TP* p_new, bool timed) {
        int tm = timed ? tic(c, PIC_T_MG) : -1;
        int n_rz = 0;
        float* z = mg_vcycle<TP>(c, (const TP*)r, a.part_rr, part_bb, part_rz, kCgBlocks, &n_rz, timed);
        toc(c, tm);
        a.p_old = p_old;
        a.p_new = p_new;
        int ta = timed ? tic(c, PIC_T_CG_A) : -1;
        if (pair)
            hipLaunchKernelGGL(k_pcg_a2, dim3(zb), dim3(kBlock), 0, c->stream, *(PcgArgs<double>*)&a,
                               (const float*)z, (const double*)part_rz, n_rz, kc);
        else
            hipLaunchKernelGGL(k_pcg_a<TP>, dim3(zb), dim3(kBlock), 0, c->stream, a, (const float*)z,
                               (const double*)part_rz, n_rz, kc);
        toc(c, ta);
        int tb = timed ? tic(c, PIC_T_CG_B) : -1;
        hipLaunchKernelGGL(k_pcg_b<TP>, dim3(kCgBlocks), dim3(kBlock), 0, c->stream, a, (const double*)part_rz, n_rz,
                           (int)zb);
        toc(c, tb);
    };
    // Without profiling, pairs of iterations run as one captured graph (the
    // kernels read the iteration state from the device, so every pair is the
    // same launch sequence; p ping-pongs p0 -> p1 -> p0 within a pair).
    hipGraph_t& graph = slot ? c->mix_graph : c->pcg_graph;
    hipGraphExec_t& exec = slot ? c->mix_exec : c->pcg_exec;
    bool use_graph = !c->prof;
    if (use_graph && !exec) {
        bool ok = true;
        if (!c->cap_stream) ok = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) == hipSuccess;
        hipStream_t keep = c->stream;
        if (ok) ok = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            c->stream = c->cap_stream;
            iteration(p0, p1, false);
            iteration(p1, p0, false);
            c->stream = keep;
            hipGraph_t gr = nullptr;
            ok = hipStreamEndCapture(c->cap_stream, &gr) == hipSuccess && gr;
            if (ok) ok = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0) == hipSuccess;
            if (ok) graph = gr;
            else if (gr) (void)hipGraphDestroy(gr);
        }
        if (!ok) {
            c->stream = keep;
            (void)hipGetLastError();
            return -2;
        }
    }
    // launch in chunks, testing convergence on the host after each; the
    // first chunk is the iteration count of the previous solve
    int chunk = c->last_iters[slot] > 2 ? c->last_iters[slot] : 2;
    int it = 0;
    while (true) {
        if (use_graph) {
            for (int t = 0; t < chunk && it <= maxit; t += 2, it += 2)
                if (hipGraphLaunch(exec, c->stream) != hipSuccess) return -2;
        } else {
            for (int t = 0; t < chunk && it <= maxit; ++t, ++it)
                iteration((it & 1) ? p1 : p0, (it & 1) ? p0 : p1, it < 64);
        }
        (void)hipMemcpyAsync(c->host_st, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream);
        if (hipStreamSynchronize(c->stream) != hipSuccess) return -2;
        if (c->host_st->done || it > maxit) break;
        chunk = 2;
    }
    c->last_iters[slot] = c->host_st->it;
    return 0;
}

int mgcg_solve(pic_ctx* c, double* phi, double V0, const int64_t* rho, int guess, double rtol, int maxit,
               pic_solve_info* info) {
    if (!c->mg_host) return -3;
    const Grid& g = c->g;
    int64_t G = (g.nn + kBlock - 1) / kBlock;
    CgArgs a;
    a.g = g;
    a.type = c->buf.node_type;
    a.x = phi;
    a.r = c->cg_r;
    a.p_old = c->cg_p0;
    a.p_new = c->cg_p1;
    a.q = c->cg_q;
    a.rho = rho;
    a.qscale = ldexp(1.0, -40) * kQe / (kEps0 * g.h);
    a.V0 = V0;
    a.V0_dev = (c->circuit && phi == c->buf.phi) ? &c->st->v_gap : nullptr;
    a.s = c->st;
    a.part_pq = c->partials + kPartPq;
    a.part_rr = c->partials + kPartRr;
    a.part_bb = c->partials + kPartBb;
    a.chunk = ((g.nn + kCgBlocks - 1) / kCgBlocks + kBlock - 1) / kBlock * kBlock;
    hipLaunchKernelGGL(k_cg_setup, dim3(1), dim3(1), 0, c->stream, c->st, rtol, maxit);
    hipLaunchKernelGGL(k_cg_init, dim3((unsigned)G), dim3(kBlock), 0, c->stream, a, guess == PIC_GUESS_ZERO);
    launch_resid(c, a);
    int e = pcg_iterate<double>(c, phi, c->cg_r, c->cg_p0, c->cg_p1, c->cg_q, maxit, 0);
    if (e) return e;
    hipLaunchKernelGGL(k_cg_zero_free, dim3((unsigned)G), dim3(kBlock), 0, c->stream, g, c->buf.node_type, phi,
                       c->st);
    (void)hipMemcpyAsync(c->host_st, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return -2;
    const DevState* h = c->host_st;
    double bn = sqrt(h->bb);
    info->iterations = h->it;
    info->relres = h->zero_solution ? 0.0 : sqrt(h->rr) / bn;
    info->relres0 = h->zero_solution ? 0.0 : sqrt(h->rr0) / bn;
    info->converged = h->zero_solution || (sqrt(h->rr) <= rtol * bn);
    return 0;
}

// ---------------------------------------------------------------------------
// Mixed precision: FP64 residual refinement around FP32 inner solves. Each
// outer step computes r = b - A phi in FP64 (k_cg_resid), solves A e = r in
// FP32 (multigrid-preconditioned CG on FP32 vectors, FP64 dot products) to a
// relative reduction of at most 1e-5, and adds e to phi in FP64.

// r32 = (float) r64, e = 0, p = 0; partials of |r32|^2 as the inner b.b and r.r
__global__ __launch_bounds__(kBlock) void k_mix_start(Grid g, const double* __restrict__ r64, float* __restrict__ r32,
                                                       float* __restrict__ e32, float* __restrict__ p32, int64_t chunk,
                                                       double* part_bb, double* part_rr) {
    int64_t b0 = xcd_block(blockIdx.x, gridDim.x) * chunk;
    int64_t b1 = b0 + chunk < g.nn ? b0 + chunk : g.nn;
    double rr = 0.0;
    for (int64_t n = b0 + threadIdx.x; n < b1; n += blockDim.x) {
        float v = (float)r64[n];
        r32[n] = v;
        e32[n] = 0.f;
        p32[n] = 0.f;
        rr += (double)v * (double)v;
    }
    __shared__ double sh[kBlock / 64];
    double t = block_sum(rr, sh);
    if (threadIdx.x == 0) {
        part_bb[blockIdx.x] = t;
        part_rr[blockIdx.x] = t;
    }
}

// phi += e (e is zero on fixed nodes)
__global__ void k_mix_update(int64_t nn, const float* __restrict__ e32, double* __restrict__ phi) {
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += (int64_t)gridDim.x * blockDim.x)
        phi[n] += (double)e32[n];
}

__global__ void k_mix_zero_free(Grid g, const uint8_t* type, double* x) {
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n < g.nn && type[n] == 0) x[n] = 0.0;
}

// outer test: FP64 r.r and b.b from the partials of k_cg_resid
__global__ void k_mix_test(const double* part_rr, const double* part_bb, DevState* s) {
    double rr = sum_partials_n(part_rr, kCgBlocks);
    double bb = sum_partials_n(part_bb, kCgBlocks);
    if (threadIdx.x == 0) {
        s->rr_outer = rr;
        s->bb = bb;
    }
}

int mixed_solve(pic_ctx* c, double* phi, double V0, const int64_t* rho, int guess, double rtol, int maxit,
                pic_solve_info* info) {
    if (!c->mg_host) return -3;
    const Grid& g = c->g;
    int64_t G = (g.nn + kBlock - 1) / kBlock;
    CgArgs a;
    a.g = g;
    a.type = c->buf.node_type;
    a.x = phi;
    a.r = c->cg_r;
    a.p_old = c->cg_p0;
    a.p_new = c->cg_p1;
    a.q = c->cg_q;
    a.rho = rho;
    a.qscale = ldexp(1.0, -40) * kQe / (kEps0 * g.h);
    a.V0 = V0;
    a.V0_dev = (c->circuit && phi == c->buf.phi) ? &c->st->v_gap : nullptr;
    a.s = c->st;
    a.part_pq = c->partials + kPartPq;
    a.part_rr = c->partials + kPartRr;
    a.part_bb = c->partials + kPartBb;
    a.chunk = ((g.nn + kCgBlocks - 1) / kCgBlocks + kBlock - 1) / kBlock * kBlock;
    // FP32 work vectors in the halves of the FP64 CG vectors (r64 stays in cg_r)
    float* r32 = (float*)c->cg_p0;
    float* e32 = r32 + g.nn;
    float* p0 = (float*)c->cg_p1;
    float* p1 = p0 + g.nn;
    float* q32 = (float*)c->cg_q;
    hipLaunchKernelGGL(k_cg_init, dim3((unsigned)G), dim3(kBlock), 0, c->stream, a, guess == PIC_GUESS_ZERO);
    int total = 0;
    double bn = 0.0, rn = 0.0, rn0 = -1.0;
    bool conv = false;
    for (int outer = 0; outer < 40; ++outer) {
        launch_resid(c, a);
        hipLaunchKernelGGL(k_mix_test, dim3(1), dim3(kBlock), 0, c->stream, (const double*)a.part_rr,
                           (const double*)a.part_bb, c->st);
        (void)hipMemcpyAsync(c->host_st, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream);
        if (hipStreamSynchronize(c->stream) != hipSuccess) return -2;
        bn = sqrt(c->host_st->bb);
        rn = sqrt(c->host_st->rr_outer);
        if (rn0 < 0) rn0 = rn;
        conv = bn == 0.0 || rn <= rtol * bn;
        if (conv || total >= maxit) break;
        // inner solve to a relative reduction that reaches rtol with a margin,
        // but not below what FP32 vectors can resolve
        double inner = std::max(1e-5, 0.5 * rtol * bn / rn);
        hipLaunchKernelGGL(k_cg_setup, dim3(1), dim3(1), 0, c->stream, c->st, inner, maxit - total);
        hipLaunchKernelGGL(k_mix_start, dim3(kCgBlocks), dim3(kBlock), 0, c->stream, g, (const double*)c->cg_r, r32,
                           e32, p0, a.chunk, a.part_bb, a.part_rr);
        int e = pcg_iterate<float>(c, e32, r32, p0, p1, q32, maxit - total, 1);
        if (e) return e;
        total += c->host_st->it;
        hipLaunchKernelGGL(k_mix_update, dim3(4096), dim3(kBlock), 0, c->stream, g.nn, (const float*)e32, phi);
    }
    info->iterations = total;
    info->relres = bn == 0.0 ? 0.0 : rn / bn;
    info->relres0 = bn == 0.0 ? 0.0 : rn0 / bn;
    info->converged = conv;
    if (bn == 0.0)
        hipLaunchKernelGGL(k_mix_zero_free, dim3((unsigned)G), dim3(kBlock), 0, c->stream, g, c->buf.node_type, phi);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// Guess of the step solve by linear extrapolation in time: with two previous
// step solves on record, phi <- 2 phi - phi_prev; phi_prev <- the old phi.
// (two nodes a thread with 16-byte accesses, one pass of the grid: every
// thread's loads are issued together)
__global__ void k_extrapolate(int64_t nn, int apply, double* __restrict__ phi, double* __restrict__ prev) {
    const int64_t n = 2 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (n + 1 < nn) {
        const double2 cur = *(const double2*)(phi + n), old = *(const double2*)(prev + n);
        if (apply) *(double2*)(phi + n) = make_double2(2.0 * cur.x - old.x, 2.0 * cur.y - old.y);
        *(double2*)(prev + n) = cur;
    } else if (n < nn) {
        const double cur = phi[n];
        if (apply) phi[n] = 2.0 * cur - prev[n];
        prev[n] = cur;
    }
}

hipError_t extrapolate_phi(pic_ctx* c, bool apply) {
    const int64_t pairs = (c->g.nn + 1) / 2;
    hipLaunchKernelGGL(k_extrapolate, dim3((unsigned)((pairs + kBlock - 1) / kBlock)), dim3(kBlock), 0, c->stream,
                       c->g.nn, apply ? 1 : 0, (double*)c->buf.phi, c->phi_prev);
    return hipGetLastError();
}

// Potential at a point by trilinear interpolation (one thread).
__global__ void k_interp(Grid g, const double* phi, double X, double Y, double Z, double* out) {
    int i = clampi((int)floor(X), 0, g.nx - 2), j = clampi((int)floor(Y), 0, g.ny - 2),
        k = clampi((int)floor(Z), 0, g.nz - 2);
    double fx = X - i, fy = Y - j, fz = Z - k;
    double s = 0.0;
    for (int t = 0; t < 8; ++t) {
        double w = ((t & 1) ? fx : 1.0 - fx) * ((t & 2) ? fy : 1.0 - fy) * ((t & 4) ? fz : 1.0 - fz);
        int64_t m = ((int64_t)(k + ((t >> 2) & 1)) * g.ny + j + ((t >> 1) & 1)) * g.nx + i + (t & 1);
        s += w * phi[m];
    }
    *out = s;
}

hipError_t apex_interp(pic_ctx* c, const double* phi, double X, double Y, double Z, double* out_dev) {
    hipLaunchKernelGGL(k_interp, dim3(1), dim3(1), 0, c->stream, c->g, phi, X, Y, Z, out_dev);
    return hipGetLastError();
}

}  // namespace pic
