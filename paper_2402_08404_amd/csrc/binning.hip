// binning.hip -- cell bins of all particles by a stable LSD radix sort of the
// cell keys (no atomics on counters, deterministic).
//
// Elements are the slots of the three species concatenated (electrons, ions,
// neutrals, each up to the slot count of the last push); the value of an
// element is species << 30 | slot and its key the tile-major cell key
// written by the push, or nkeys for a removed particle (sorted last). Each
// pass sorts by 8 bits: per-tile digit histograms, a scan of the histograms
// in digit-major order, then a stable scatter in which every element finds
// its rank among equal digits of its tile with wavefront ballots. After the
// last pass, off[c] is the first position of key c (a lower bound found from
// the sorted keys), so bins[off[c] .. off[c+1]) are the particles of cell c.
#include "pic_internal.hpp"

namespace pic {

constexpr int kSortItems = 16;
constexpr int kSortTile = kBlock * kSortItems;  // elements per block
constexpr int kRadix = 256;

struct SortIn {
    const uint32_t* key[3];   // per-species keys (pass 0)
    const uint32_t* kin;      // keys of passes >= 1
    const uint32_t* vin;      // values of passes >= 1
    const DevState* st;
};

__device__ inline int64_t total_elems(const DevState* st) {
    return (int64_t)(st->n_push[0] + st->n_push[1] + st->n_push[2]);
}

// key and value of element e in pass 0 (straight from the species arrays)
__device__ inline void elem0(const SortIn& in, int64_t e, uint32_t nkeys, uint32_t& k, uint32_t& v) {
    int64_t n0 = (int64_t)in.st->n_push[0], n1 = (int64_t)in.st->n_push[1];
    int s;
    int64_t i;
    if (e < n0) {
        s = 0;
        i = e;
    } else if (e < n0 + n1) {
        s = 1;
        i = e - n0;
    } else {
        s = 2;
        i = e - n0 - n1;
    }
    k = in.key[s][i];
    if (k == kDead) k = nkeys;
    v = ((uint32_t)s << 30) | (uint32_t)i;
}

__device__ inline void elem(const SortIn& in, int pass, int64_t e, uint32_t nkeys, uint32_t& k, uint32_t& v) {
    if (pass == 0) {
        elem0(in, e, nkeys, k, v);
    } else {
        k = in.kin[e];
        v = in.vin[e];
    }
}

// Per-tile digit histogram, stored digit-major: hist[d * nb + b].
__global__ __launch_bounds__(kBlock) void k_rs_hist(SortIn in, int pass, uint32_t nkeys, uint32_t* hist, int64_t nb) {
    __shared__ uint32_t h[kRadix];
    int64_t n = total_elems(in.st);
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kSortTile;
    int shift = 8 * pass;
    for (int r = 0; r < kSortItems; ++r) {
        int64_t e = base + r * kBlock + threadIdx.x;
        if (e < n) {
            uint32_t k, v;
            elem(in, pass, e, nkeys, k, v);
            atomicAdd(&h[(k >> shift) & 255u], 1u);
        }
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: rank among equal digits within the tile (rounds of 256
// elements in order; inside a round, lower threads first).
__global__ __launch_bounds__(kBlock) void k_rs_scatter(SortIn in, int pass, uint32_t nkeys, const uint32_t* hoff,
                                                       int64_t nb, uint32_t* kout, uint32_t* vout) {
    __shared__ uint32_t base_d[kRadix];      // global offset of each digit for this tile
    __shared__ uint32_t wcnt[kBlock / 64][kRadix];
    int64_t n = total_elems(in.st);
    base_d[threadIdx.x] = hoff[(int64_t)threadIdx.x * nb + blockIdx.x];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int shift = 8 * pass;
    int64_t tbase = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; ++r) {
        for (int q = 0; q < kBlock / 64; ++q) wcnt[q][threadIdx.x] = 0;
        __syncthreads();
        int64_t e = tbase + r * kBlock + threadIdx.x;
        bool valid = e < n;
        uint32_t k = 0, v = 0, d = 0;
        if (valid) {
            elem(in, pass, e, nkeys, k, v);
            d = (k >> shift) & 255u;
        }
        // lanes of this wavefront with the same digit
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t m = __ballot(valid && ((d >> b) & 1u));
            same &= ((d >> b) & 1u) ? m : ~m;
        }
        uint32_t rank_w = (uint32_t)__popcll(same & lt);
        if (valid && rank_w == 0) wcnt[w][d] = (uint32_t)__popcll(same);
        __syncthreads();
        if (valid) {
            uint32_t pos = base_d[d] + rank_w;
            for (int q = 0; q < w; ++q) pos += wcnt[q][d];
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int q = 0; q < kBlock / 64; ++q) add += wcnt[q][threadIdx.x];
        base_d[threadIdx.x] += add;
        __syncthreads();
    }
}

// Per-key counts of the sorted keys (integer atomics: the counts, and so the
// offsets, do not depend on the order of the increments). Removed particles
// (key nkeys, sorted last) are not counted: no offset needs them.
__global__ void k_rs_count(const uint32_t* __restrict__ keys, const DevState* st, uint32_t nkeys,
                           uint32_t* __restrict__ cnt) {
    int64_t n = total_elems(st);
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        const uint32_t k = keys[p];
        if (k < nkeys) atomicAdd(&cnt[k], 1u);
    }
}

// off[c] = first position whose key is >= c, for c = 0 .. nkeys (binary
// search in the sorted keys; bounded work per cell whatever the gaps).
__global__ void k_rs_offsets(const uint32_t* __restrict__ keys, const DevState* st, uint32_t nkeys,
                             uint32_t* __restrict__ off) {
    int64_t n = total_elems(st);
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= (int64_t)nkeys; c += stride) {
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if ((int64_t)keys[mid] < c) lo = mid + 1;
            else hi = mid;
        }
        off[c] = (uint32_t)lo;
    }
}

// Sort the keys of the last push into c->bins / c->off. Work buffers: the
// per-species key arrays are the pass-0 input; two ping-pong pairs of
// (key, value) arrays of sum(cap) elements; the digit histograms.
hipError_t radix_bins(pic_ctx* c) {
    int64_t capsum = c->buf.cap[0] + c->buf.cap[1] + c->buf.cap[2];
    int64_t nb = (capsum + kSortTile - 1) / kSortTile;
    if (nb < 1) nb = 1;
    uint32_t nkeys = (uint32_t)c->g.nkeys;
    int passes = 0;
    for (uint64_t m = (uint64_t)nkeys; m > 0; m >>= 8) ++passes;  // keys are 0..nkeys
    SortIn in;
    for (int s = 0; s < 3; ++s) in.key[s] = c->key[s];
    in.st = c->st;
    uint32_t* kbuf[2] = {c->rs_keys[0], c->rs_keys[1]};
    uint32_t* vbuf[2] = {c->rs_vals[0], c->rs_vals[1]};
    // the last pass must land in c->bins
    int out_idx = (passes - 1) & 1;
    vbuf[out_idx] = c->bins;
    for (int p = 0; p < passes; ++p) {
        in.kin = kbuf[(p + 1) & 1];
        in.vin = vbuf[(p + 1) & 1];
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nb), dim3(kBlock), 0, c->stream, in, p, nkeys, c->rs_hist, nb);
        hipError_t e = scan_u32(c, c->rs_hist, c->rs_hist, (int64_t)kRadix * nb, nullptr, nullptr, false, false);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nb), dim3(kBlock), 0, c->stream, in, p, nkeys, c->rs_hist, nb,
                           kbuf[p & 1], vbuf[p & 1]);
    }
    // off = exclusive scan of the per-key counts (keys 0 .. nkeys, the last
    // one counting removed particles)
    hipError_t e = launch_zero(c->off, ((size_t)nkeys + 1) * 4, c->stream);
    if (e != hipSuccess) return e;
    int64_t Gc = (capsum + kBlock - 1) / kBlock;
    if (Gc > 16384) Gc = 16384;
    if (Gc < 1) Gc = 1;
    hipLaunchKernelGGL(k_rs_count, dim3((unsigned)Gc), dim3(kBlock), 0, c->stream, (const uint32_t*)kbuf[out_idx],
                       (const DevState*)c->st, nkeys, c->off);
    e = scan_u32(c, c->off, c->off, (int64_t)nkeys + 1, nullptr, nullptr, false, false);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace pic
