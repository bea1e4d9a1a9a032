// binning.hip -- cell bins of all particles by a counting sort of the cell
// keys.
//
// Elements are the slots of the three species concatenated (electrons, ions,
// neutrals, each up to the slot count of the last push); the value of an
// element is species << 30 | slot and its key the tile-major cell key
// written by the push (removed particles carry no key and are left out).
// Counts per key by integer atomics, their exclusive scan gives off[c], and
// a scatter through per-key cursors puts every element in its bin, so
// bins[off[c] .. off[c+1]) are the particles of cell c and off[nkeys] is the
// number of live particles. The counts, the offsets and the set of elements
// of every bin do not depend on the order of the atomics; the order inside a
// bin does, and nothing relies on it: the collision kernels order each cell
// by (species, id) and write that order back before the arrays are
// reordered, and the deposit adds integers. In both passes the lanes of a
// wavefront holding a run of equal keys (the arrays are kept nearly in cell
// order) issue one atomic for the whole run.
#include "pic_internal.hpp"

namespace pic {

__device__ inline int64_t total_elems(const DevState* st) {
    return (int64_t)(st->n_push[0] + st->n_push[1] + st->n_push[2]);
}

// key (kDead if none) and value of element e
__device__ inline void elem_kv(const uint32_t* const key[3], const DevState* st, int64_t e, uint32_t& k, uint32_t& v) {
    const int64_t n0 = (int64_t)st->n_push[0], n1 = (int64_t)st->n_push[1];
    const int s = e < n0 ? 0 : (e < n0 + n1 ? 1 : 2);
    const int64_t i = e - (s >= 1 ? n0 : 0) - (s == 2 ? n1 : 0);
    k = key[s][i];
    v = ((uint32_t)s << 30) | (uint32_t)i;
}

struct BinIn {
    const uint32_t* key[3];
    const DevState* st;
    uint32_t nkeys;
};

// Runs of equal keys inside a wavefront: the run's first lane (head), the
// run length (at the head) and every lane's offset inside its run.
struct Run {
    bool head;
    int first, len;
};

__device__ inline Run wave_run(uint32_t k) {
    const int lane = threadIdx.x & 63;
    const uint32_t kp = __shfl_up(k, 1);
    const bool head = lane == 0 || k != kp;
    const unsigned long long heads = __ballot(head);
    Run r;
    r.head = head;
    // first = the highest head at or below this lane
    const unsigned long long below = heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1));
    r.first = 63 - __clzll(below);
    // len (valid at a head) = distance to the next head, or to the wave end
    const unsigned long long above = lane == 63 ? 0ull : (heads & ~((2ull << lane) - 1));
    const int next = above ? __ffsll((long long)above) - 1 : 64;
    r.len = next - lane;
    return r;
}

// cnt[k] += number of live elements with key k
__global__ __launch_bounds__(kBlock) void k_bin_count(BinIn in, uint32_t* __restrict__ cnt) {
    const int64_t n = total_elems(in.st);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x; b < n; b += stride) {
        const int64_t e = b + threadIdx.x;
        uint32_t k = kDead, v = 0;
        if (e < n) elem_kv(in.key, in.st, e, k, v);
        if (k >= in.nkeys) k = kDead;
        const Run r = wave_run(k);
        if (r.head && k != kDead) atomicAdd(&cnt[k], (uint32_t)r.len);
    }
}

// bins[cursor[k]++] = value, one atomic per run of equal keys
__global__ __launch_bounds__(kBlock) void k_bin_scatter(BinIn in, uint32_t* __restrict__ cursor,
                                                         uint32_t* __restrict__ bins) {
    const int64_t n = total_elems(in.st);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int lane = threadIdx.x & 63;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x; b < n; b += stride) {
        const int64_t e = b + threadIdx.x;
        uint32_t k = kDead, v = 0;
        if (e < n) elem_kv(in.key, in.st, e, k, v);
        if (k >= in.nkeys) k = kDead;
        const Run r = wave_run(k);
        uint32_t base = 0;
        if (r.head && k != kDead) base = atomicAdd(&cursor[k], (uint32_t)r.len);
        base = __shfl(base, r.first);
        if (k != kDead) bins[base + (uint32_t)(lane - r.first)] = v;
    }
}

__global__ void k_copy_u32(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = in[i];
}

// Bins of the keys of the last push into c->bins / c->off; c->cursor is the
// scatter's work array (nkeys entries).
hipError_t cell_bins(pic_ctx* c) {
    const int64_t capsum = c->buf.cap[0] + c->buf.cap[1] + c->buf.cap[2];
    const uint32_t nkeys = (uint32_t)c->g.nkeys;
    BinIn in;
    for (int s = 0; s < 3; ++s) in.key[s] = c->key[s];
    in.st = c->st;
    in.nkeys = nkeys;
    int64_t G = (capsum + kBlock - 1) / kBlock;
    if (G > 16384) G = 16384;
    if (G < 1) G = 1;
    hipError_t e = launch_zero(c->off, ((size_t)nkeys + 1) * 4, c->stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_count, dim3((unsigned)G), dim3(kBlock), 0, c->stream, in, c->off);
    e = scan_u32(c, c->off, c->off, (int64_t)nkeys + 1, nullptr, nullptr, false, false);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_copy_u32, dim3(4096), dim3(kBlock), 0, c->stream, (const uint32_t*)c->off, c->cursor,
                       (int64_t)nkeys);
    hipLaunchKernelGGL(k_bin_scatter, dim3((unsigned)G), dim3(kBlock), 0, c->stream, in, c->cursor, c->bins);
    return hipGetLastError();
}

}  // namespace pic
