// binning.hip -- cell bins of all particles by a counting sort of the cell
// keys, without a global atomic per particle.
//
// Elements are the slots of the three species (electrons, ions, neutrals,
// each up to the slot count of the push); the value of an element is
// species << 30 | slot (stored with the particle's id, so that the collision
// kernels read the ids in cell order), its key the tile-major cell key
// written by the push (removed particles carry no key and are left out).
// Keys are grouped: a group is 2^s consecutive tiles of 8^3 cells (s the
// smallest that leaves at most kBinTargetGroups groups, up to 8 tiles), and
// the slots are cut into chunks of kBinChunk per species. Few large groups
// keep the scattered writes of a chunk contiguous within each group (about
// kBinChunk / groups records in a row). The sort runs in two levels:
//  1. k_bin_hist: per chunk, a histogram over the groups in LDS (LDS
//     atomics), written per chunk;
//  2. k_bin_colscan / k_bin_segscan: per group, exclusive prefix sums over
//     the chunks (in segments, then across segments) and the group totals;
//     an exclusive scan of the totals gives every group's first bin;
//  3. k_bin_group_place: per chunk, the group counters in LDS start at the
//     chunk's place in each group, and every element takes the next one (an
//     LDS atomic), writing {value, id, cell index within the group} to a
//     staging array in group order (one 16-byte store);
//  4. k_bin_cells: per group, an LDS counting sort by cell gives off[c] of
//     the group's cells and moves the elements into bins in cell order.
// bins[off[c] .. off[c+1]) are then the particles of cell c and off[nkeys]
// the number of live particles. Counts, offsets and the set of elements of a
// bin do not depend on the order of the atomics; the order inside a bin
// does, and nothing relies on it: the collision kernels order each cell by
// (species, id) and write that order back before the arrays are reordered,
// and the deposit adds integers.
#include "pic_internal.hpp"

namespace pic {

constexpr int kBinThreads = 512;
constexpr int kBinUnroll = 8;
constexpr int kBinCellsPer = 16;                          // elements per thread held in registers
constexpr int kBinCellsRegs = kBinCellsPer * kBinThreads;  // largest group sorted in one read

// Runs of equal values inside a wavefront (all 64 lanes take part): the
// run's first lane and, at that lane (the head), the run length. Slots in
// order of the cells come in long runs, so one LDS atomic per run replaces
// up to 64 atomics on one address.
struct Run {
    bool head;
    int first, len;
};

__device__ inline Run wave_run(uint32_t k) {
    const int lane = threadIdx.x & 63;
    const uint32_t kp = __shfl_up(k, 1, 64);
    const bool head = lane == 0 || k != kp;
    const unsigned long long heads = __ballot(head);
    Run r;
    r.head = head;
    const unsigned long long below = heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1));
    r.first = 63 - __clzll(below);
    const unsigned long long above = lane == 63 ? 0ull : (heads & ~((2ull << lane) - 1));
    const int next = above ? __ffsll((long long)above) - 1 : 64;
    r.len = next - lane;
    return r;
}

// h[k] += 1 for every lane with k != kDead (one atomic per run)
__device__ inline void lds_count(uint32_t* h, uint32_t k) {
    const Run r = wave_run(k);
    if (r.head && k != kDead) atomicAdd(&h[k], (uint32_t)r.len);
}

// the lane's place: h[k] before its run plus its place in the run, h[k]
// advanced by the run (undefined for k == kDead)
__device__ inline uint32_t lds_take(uint32_t* h, uint32_t k) {
    const Run r = wave_run(k);
    uint32_t base = 0;
    if (r.head && k != kDead) base = atomicAdd(&h[k], (uint32_t)r.len);
    base = __shfl(base, r.first, 64);
    return base + (uint32_t)((int)(threadIdx.x & 63) - r.first);
}

struct BinArgs {
    const uint32_t* key[3];
    const uint32_t* id[3];
    const DevState* st;
    uint32_t nkeys;
    int ng;              // groups
    int gshift;          // log2 of the cells per group
    int nchunk[3];       // chunks per species
    int nchunk_all;
    int nseg;            // segments of the chunk range in the column scan
    uint32_t* hist;      // [chunk][group] counts, then exclusive prefixes within a segment
    uint32_t* segtot;    // [segment][group] totals, then exclusive prefixes across segments
    uint32_t* gbase;     // [group] totals, then first bins (ng + 1 entries)
    uint4* stage;        // elements in group order: {value, id, cell index within the group, 0}
    uint2* bins;
    uint32_t* off;
};

// species and slot range of chunk b (empty past the push's slots)
__device__ inline void chunk_range(const BinArgs& a, int b, int& s, int64_t& i0, int64_t& i1) {
    s = b < a.nchunk[0] ? 0 : (b < a.nchunk[0] + a.nchunk[1] ? 1 : 2);
    const int j = b - (s >= 1 ? a.nchunk[0] : 0) - (s == 2 ? a.nchunk[1] : 0);
    const int64_t n = (int64_t)a.st->n_push[s];
    i0 = (int64_t)j * kBinChunk;
    i1 = i0 + kBinChunk < n ? i0 + kBinChunk : n;
}

__global__ __launch_bounds__(kBinThreads) void k_bin_hist(BinArgs a) {
    extern __shared__ uint32_t h[];  // ng counters
    for (int g = threadIdx.x; g < a.ng; g += kBinThreads) h[g] = 0u;
    __syncthreads();
    int s;
    int64_t i0, i1;
    chunk_range(a, (int)blockIdx.x, s, i0, i1);
    const uint32_t* __restrict__ key = a.key[s];
    // kBinUnroll keys per thread are loaded before their atomics
    for (int64_t b0 = i0; b0 < i1; b0 += kBinUnroll * kBinThreads) {
        uint32_t k[kBinUnroll];
#pragma unroll
        for (int u = 0; u < kBinUnroll; ++u) {
            const int64_t i = b0 + u * kBinThreads + threadIdx.x;
            k[u] = i < i1 ? key[i] : kDead;
        }
#pragma unroll
        for (int u = 0; u < kBinUnroll; ++u) lds_count(h, k[u] < a.nkeys ? k[u] >> a.gshift : kDead);
    }
    __syncthreads();
    uint32_t* out = a.hist + (int64_t)blockIdx.x * a.ng;
    for (int g = threadIdx.x; g < a.ng; g += kBinThreads) out[g] = h[g];
}

// thread (segment, group): exclusive prefixes over the segment's chunks
__global__ __launch_bounds__(kBlock) void k_bin_colscan(BinArgs a) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)a.nseg * a.ng) return;
    const int g = (int)(t % a.ng), seg = (int)(t / a.ng);
    const int per = (a.nchunk_all + a.nseg - 1) / a.nseg;
    const int c0 = seg * per, c1 = c0 + per < a.nchunk_all ? c0 + per : a.nchunk_all;
    uint32_t run = 0;
    for (int cc = c0; cc < c1; ++cc) {
        uint32_t* q = a.hist + (int64_t)cc * a.ng + g;
        const uint32_t v = *q;
        *q = run;
        run += v;
    }
    a.segtot[(int64_t)seg * a.ng + g] = run;
}

// thread per group: exclusive prefixes across segments, and the group total
__global__ __launch_bounds__(kBlock) void k_bin_segscan(BinArgs a) {
    const int g = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (g >= a.ng) return;
    uint32_t run = 0;
    for (int seg = 0; seg < a.nseg; ++seg) {
        uint32_t* q = a.segtot + (int64_t)seg * a.ng + g;
        const uint32_t v = *q;
        *q = run;
        run += v;
    }
    a.gbase[g] = run;
}

__global__ __launch_bounds__(kBinThreads) void k_bin_group_place(BinArgs a) {
    extern __shared__ uint32_t h[];  // ng counters
    const int b = (int)blockIdx.x;
    const int per = (a.nchunk_all + a.nseg - 1) / a.nseg;
    const uint32_t* segp = a.segtot + (int64_t)(b / per) * a.ng;
    const uint32_t* hp = a.hist + (int64_t)b * a.ng;
    for (int g = threadIdx.x; g < a.ng; g += kBinThreads) h[g] = a.gbase[g] + segp[g] + hp[g];
    __syncthreads();
    int s;
    int64_t i0, i1;
    chunk_range(a, b, s, i0, i1);
    const uint32_t* __restrict__ key = a.key[s];
    const uint32_t* __restrict__ id = a.id[s];
    const uint32_t cmask = (1u << a.gshift) - 1u;
    for (int64_t b0 = i0; b0 < i1; b0 += kBinUnroll * kBinThreads) {
        uint32_t k[kBinUnroll], v[kBinUnroll];
#pragma unroll
        for (int u = 0; u < kBinUnroll; ++u) {
            const int64_t i = b0 + u * kBinThreads + threadIdx.x;
            k[u] = i < i1 ? key[i] : kDead;
            v[u] = i < i1 ? id[i] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kBinUnroll; ++u) {
            const bool ok = k[u] < a.nkeys;
            const uint32_t d = lds_take(h, ok ? k[u] >> a.gshift : kDead);
            if (!ok) continue;
            const uint32_t i = (uint32_t)(b0 + u * kBinThreads + threadIdx.x);
            a.stage[d] = make_uint4(((uint32_t)s << 30) | i, v[u], k[u] & cmask, 0u);
        }
    }
}

// exclusive scan of cnt[0 .. cpg) in place, starting at e0: each thread a
// run of cpg / kBinThreads cells, then the runs across the block
__device__ inline void cells_scan(uint32_t* cnt, uint32_t* wsum, int cpg, uint32_t e0) {
    const int R = cpg / kBinThreads;
    uint32_t loc = 0;
    for (int r = 0; r < R; ++r) loc += cnt[threadIdx.x * R + r];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = loc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(inc, o, 64);
        if (lane >= o) inc += v;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t run = e0 + inc - loc;
    for (int q = 0; q < w; ++q) run += wsum[q];
    for (int r = 0; r < R; ++r) {
        const int j = threadIdx.x * R + r;
        const uint32_t v = cnt[j];
        cnt[j] = run;
        run += v;
    }
    __syncthreads();
}

// One block per group: counting sort of the group's elements by cell. A
// group of at most kBinCellsRegs elements is read once: each element takes
// its rank within its cell while counting and waits in registers for the
// scan; a larger group is read twice (count, then place).
__global__ __launch_bounds__(kBinThreads) void k_bin_cells(BinArgs a) {
    __shared__ uint32_t cnt[kBinMaxCellsPerGroup];
    __shared__ uint32_t wsum[kBinThreads / 64];
    const int g = (int)blockIdx.x;
    const int cpg = 1 << a.gshift;
    const uint32_t e0 = a.gbase[g], e1 = a.gbase[g + 1];
    for (int j = threadIdx.x; j < cpg; j += kBinThreads) cnt[j] = 0u;
    __syncthreads();
    const int64_t key0 = (int64_t)g << a.gshift;
    if (e1 - e0 <= (uint32_t)kBinCellsRegs) {
        uint4 v[kBinCellsPer];
        uint32_t rk[kBinCellsPer];
#pragma unroll
        for (int u = 0; u < kBinCellsPer; ++u) {
            const uint32_t e = e0 + u * kBinThreads + threadIdx.x;
            v[u] = e < e1 ? a.stage[e] : make_uint4(0u, 0u, kDead, 0u);
        }
#pragma unroll
        for (int u = 0; u < kBinCellsPer; ++u) rk[u] = lds_take(cnt, v[u].z);
        __syncthreads();
        cells_scan(cnt, wsum, cpg, e0);
        for (int j = threadIdx.x; j < cpg; j += kBinThreads)
            if (key0 + j < (int64_t)a.nkeys) a.off[key0 + j] = cnt[j];
#pragma unroll
        for (int u = 0; u < kBinCellsPer; ++u)
            if (v[u].z != kDead) a.bins[cnt[v[u].z] + rk[u]] = make_uint2(v[u].x, v[u].y);
    } else {
        for (uint32_t b = e0; b < e1; b += kBinThreads) {
            const uint32_t e = b + threadIdx.x;
            lds_count(cnt, e < e1 ? a.stage[e].z : kDead);
        }
        __syncthreads();
        cells_scan(cnt, wsum, cpg, e0);
        for (int j = threadIdx.x; j < cpg; j += kBinThreads)
            if (key0 + j < (int64_t)a.nkeys) a.off[key0 + j] = cnt[j];
        __syncthreads();
        for (uint32_t b = e0; b < e1; b += kBinThreads) {
            const uint32_t e = b + threadIdx.x;
            const uint4 v = e < e1 ? a.stage[e] : make_uint4(0u, 0u, kDead, 0u);
            const uint32_t d = lds_take(cnt, v.z);
            if (e < e1) a.bins[d] = make_uint2(v.x, v.y);
        }
    }
    if (g == a.ng - 1 && threadIdx.x == 0) a.off[a.nkeys] = e1;
}

// Bins of the keys of the last push into c->bins / c->off.
hipError_t cell_bins(pic_ctx* c) {
    BinArgs a;
    for (int s = 0; s < 3; ++s) {
        a.key[s] = c->key[s];
        a.id[s] = c->buf.id[s];
        a.nchunk[s] = (int)((c->buf.cap[s] + kBinChunk - 1) / kBinChunk);
    }
    a.st = c->st;
    a.nkeys = (uint32_t)c->g.nkeys;
    a.gshift = c->bin_gshift;
    a.ng = c->bin_ng;
    a.nchunk_all = a.nchunk[0] + a.nchunk[1] + a.nchunk[2];
    a.nseg = kBinSegments;
    a.hist = c->bin_hist;
    a.segtot = c->bin_segtot;
    a.gbase = c->bin_gbase;
    a.stage = c->bin_stage;
    a.bins = c->bins;
    a.off = c->off;
    if (a.nchunk_all == 0) return hipSuccess;
    const size_t lds = (size_t)a.ng * 4;
    hipLaunchKernelGGL(k_bin_hist, dim3((unsigned)a.nchunk_all), dim3(kBinThreads), lds, c->stream, a);
    const int64_t ncol = (int64_t)a.nseg * a.ng;
    hipLaunchKernelGGL(k_bin_colscan, dim3((unsigned)((ncol + kBlock - 1) / kBlock)), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL(k_bin_segscan, dim3((unsigned)((a.ng + kBlock - 1) / kBlock)), dim3(kBlock), 0, c->stream, a);
    hipError_t e = scan_u32(c, a.gbase, a.gbase, a.ng, nullptr, a.gbase + a.ng, false, false);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_group_place, dim3((unsigned)a.nchunk_all), dim3(kBinThreads), lds, c->stream, a);
    hipLaunchKernelGGL(k_bin_cells, dim3((unsigned)a.ng), dim3(kBinThreads), 0, c->stream, a);
    return hipGetLastError();
}

}  // namespace pic
