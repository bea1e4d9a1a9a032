// binning.hip -- cell bins of all particles by a counting sort of the cell
// keys.
//
// Elements are the slots of the three species concatenated (electrons, ions,
// neutrals, each up to the slot count of the last push); the value of an
// element is species << 30 | slot (stored with the particle's id, so that the
// collision kernels read the ids in cell order) and its key the tile-major cell key
// written by the push (removed particles carry no key and are left out).
// The push counts the keys by integer atomics into off (count_key, one
// atomic per run of equal keys in a wavefront: the arrays are kept nearly in
// cell order) and keeps each particle's rank among those of its key; the
// exclusive scan of the counts gives off[c], and every element goes to
// bins[off[key] + rank], so bins[off[c] .. off[c+1]) are the particles of
// cell c and off[nkeys] is the number of live particles. The counts, the
// offsets and the set of elements of every bin do not depend on the order of
// the atomics; the order inside a bin does, and nothing relies on it: the
// collision kernels order each cell by (species, id) and write that order
// back before the arrays are reordered, and the deposit adds integers.
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
    const uint32_t* id[3];
    const uint32_t* rank[3];  // rank of each slot among the particles of its key (from the push)
    const DevState* st;
    uint32_t nkeys;
};

// bins[off[k] + rank] = {value, id} for every element with a key k
__global__ __launch_bounds__(kBlock) void k_bin_place(BinIn in, const uint32_t* __restrict__ off,
                                                       uint2* __restrict__ bins) {
    const int64_t n = total_elems(in.st);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        uint32_t k, v;
        elem_kv(in.key, in.st, e, k, v);
        if (k >= in.nkeys) continue;
        const int s = (int)(v >> 30);
        const uint32_t i = v & 0x3FFFFFFFu;
        bins[off[k] + in.rank[s][i]] = make_uint2(v, in.id[s][i]);
    }
}

// Bins of the keys of the last push into c->bins / c->off (holding the
// counts of the push, and c->rank the ranks).
hipError_t cell_bins(pic_ctx* c) {
    const int64_t capsum = c->buf.cap[0] + c->buf.cap[1] + c->buf.cap[2];
    const uint32_t nkeys = (uint32_t)c->g.nkeys;
    BinIn in;
    for (int s = 0; s < 3; ++s) {
        in.key[s] = c->key[s];
        in.id[s] = c->buf.id[s];
        in.rank[s] = c->rank + (s >= 1 ? c->buf.cap[0] : 0) + (s == 2 ? c->buf.cap[1] : 0);
    }
    in.st = c->st;
    in.nkeys = nkeys;
    int64_t G = (capsum + kBlock - 1) / kBlock;
    if (G > 16384) G = 16384;
    if (G < 1) G = 1;
    hipError_t e = scan_u32(c, c->off, c->off, (int64_t)nkeys + 1, nullptr, nullptr, false, false);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_place, dim3((unsigned)G), dim3(kBlock), 0, c->stream, in, (const uint32_t*)c->off,
                       c->bins);
    return hipGetLastError();
}

}  // namespace pic
