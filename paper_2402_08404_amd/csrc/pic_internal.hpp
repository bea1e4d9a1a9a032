// pic_internal.hpp -- types and device helpers shared by the libpic kernels.
//
// Particle state is SoA per species in grid units (X = x/h, V = v dt/h);
// node arrays are x-fastest, index n = (k*ny + j)*nx + i; cell (i,j,k) spans
// nodes i..i+1, j..j+1, k..k+1 and has index (k*(ny-1) + j)*(nx-1) + i.
#pragma once

#include <vector>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "pic.h"

namespace pic {

// CODATA 2022 (SI).
constexpr double kQe = 1.602176634e-19;
constexpr double kMe = 9.1093837139e-31;
constexpr double kEps0 = 8.8541878188e-12;
constexpr double kHpl = 6.62607015e-34;
constexpr double kPi = 3.14159265358979323846;

constexpr uint32_t kDead = 0xFFFFFFFFu;      // id of a free slot, key of a removed particle
constexpr int kSmallCell = 16;                // cells up to this many particles: one thread each
constexpr int kMidCell = 256;                 // listed cells up to this many: a small-LDS wavefront each
constexpr int kBigCell = 4096;                // cells up to this many: one wavefront each
constexpr int kBlock = 256;

// Third Philox counter word: purpose of the draw.
constexpr uint32_t kTagMcc1 = 1, kTagMcc2 = 2, kTagPair1 = 3, kTagPair2 = 4, kTagFi = 5, kTagInj = 6, kTagEvap = 7;
// added to a tag for the draws of the second and later sub-particles of a
// weighted superparticle (sub-particle q >= 1 draws with counter word q)
constexpr uint32_t kTagSub = 16;
// same-species and Coulomb pairing: cell shifts (Cu-Cu, e-e, Cu+-Cu+, e-Cu+)
// and pair draws (Cu-Cu, same-species Coulomb, e-Cu+ Coulomb)
constexpr uint32_t kTagPairNN = 8, kTagNN = 9, kTagPairEE = 10, kTagPairII = 11, kTagPairEI = 12, kTagCoul = 13,
                   kTagCoulEI = 14;
// recombination: cell shift and pair draws
constexpr uint32_t kTagPairRec = 32, kTagRec = 33;

// Device-resident counters and scalars of one context.
struct DevState {
    unsigned long long n_slots[3];
    unsigned long long n_push[3];      // slots covered by the bins of the last push/deposit
    unsigned long long next_id;
    unsigned long long absorbed[3][5];
    unsigned long long events[5];
    unsigned long long injected, fn_clamped, bsi_count;
    unsigned long long n_fi, n_prod, n_prod_kind[2], n_ev, n_big;
    unsigned long long n_sorted[3];
    double fn_expected;
    unsigned int smax_bits[3];         // max |V| per species (float bits, rounded up)
    int error;
    // CG scalars
    double rr, bb, rr0, pq, alpha, beta, rtol;
    double rrbuf[2], rzbuf[2];
    double rz_prev;                    // r.z of the previous preconditioned iteration
    int it, maxit, done, zero_solution;
    unsigned int red_count;
    // mixed-precision refinement
    double rr_outer;
    // learned warm start: s = max |q| of the current charge; gamma = the
    // weight of the network output y in the guess V0 phi1 + gamma y
    double learn_scale;
    double learn_gamma;
    int learn_bad;                     // the network output of the last learned guess was not finite
    // surface and circuit terms
    unsigned long long evaporated;
    double evap_expected;
    double bomb_e[2];                  // kinetic energy of ions absorbed at the cathode plane / the tip [J]
    double isr[2];                     // Shockley-Ramo current of the last push, electrons and ions [A]
    double v_gap, i_gap, i_tot;        // RC circuit: gap voltage (anode potential), currents [V, A]
    // superparticle weights
    unsigned long long events_w[5];    // physical collisions per kind (sum of N_coll)
    unsigned long long n_split[3];     // superparticles split off in this collide phase, per species
    unsigned long long splits;         // cumulative split-offs
    unsigned long long evap_atoms;     // cumulative evaporated atoms
    unsigned long long merges[3];      // cumulative merged pairs per species
    unsigned long long nn_events;      // cumulative Cu-Cu elastic collisions
    unsigned long long coulomb_pairs;  // cumulative Coulomb scatterings
    unsigned long long n_rec;          // recombinations of this collide phase
    unsigned long long recombinations; // cumulative recombinations
    unsigned long long n_big2;         // listed cells of more than kMidCell particles (from the list's end)
};

// Cells are numbered tile-major: tiles of kTile^3 cells, tile index
// (tz*nty + ty)*ntx + tx, then the cell inside the tile (lz*kTile + ly)*kTile
// + lx. nkeys = ntiles * kTile^3 >= nc (edge tiles may be partial).
constexpr int kTile = 8;
constexpr int kTileCells = kTile * kTile * kTile;
// binning (binning.hip): slots per chunk, wanted and largest group count
// (the LDS histogram of a chunk), largest group in cells, segments of the
// column scan
constexpr int kBinChunk = 32768;
constexpr int kBinTargetGroups = 4096;
constexpr int kBinMaxGroups = 16384;
constexpr int kBinMaxCellsPerGroup = 4096;
constexpr int kBinSegments = 32;

struct Grid {
    int nx, ny, nz;
    double h, R, H, zc, xc, yc;
    int64_t nn, nc;
    int ntx, nty, ntz;
    int64_t nkeys;
};

__host__ __device__ inline uint32_t cell_key(const Grid& g, int i, int j, int k) {
    int tx = i / kTile, ty = j / kTile, tz = k / kTile;
    uint32_t tile = (uint32_t)((tz * g.nty + ty) * g.ntx + tx);
    return tile * (uint32_t)kTileCells + (uint32_t)(((k % kTile) * kTile + (j % kTile)) * kTile + (i % kTile));
}

// Cell (i, j, k) of a key; the linear cell index is (k*(ny-1) + j)*(nx-1) + i.
__host__ __device__ inline void key_cell(const Grid& g, uint32_t key, int& i, int& j, int& k) {
    uint32_t tile = key / kTileCells, l = key % kTileCells;
    int tx = (int)(tile % g.ntx), ty = (int)((tile / g.ntx) % g.nty), tz = (int)(tile / (g.ntx * g.nty));
    i = tx * kTile + (int)(l % kTile);
    j = ty * kTile + (int)((l / kTile) % kTile);
    k = tz * kTile + (int)(l / (kTile * kTile));
}

template <typename T>
struct Species {
    T *x, *y, *z, *vx, *vy, *vz;
    uint32_t* id;
    int64_t cap;
    uint32_t* w;   // superparticle weights (null: every weight is 1)
};

template <typename T>
struct V4 {};
template <>
struct V4<float> { using type = float4; };
template <>
struct V4<double> { using type = double4; };

// ---------------------------------------------------------------------------
// Device helpers

// Philox4x32-10 (Salmon et al., SC'11).
__device__ inline void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint32_t hi0 = __umulhi(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
        uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
        uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// Uniform in (0,1) from 52 bits: (k + 1/2) 2^-52, exact in FP64.
__device__ inline double u52(uint32_t hi, uint32_t lo) {
    uint64_t k = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
    return ((double)k + 0.5) * 0x1p-52;
}

struct Draw2 { double a, b; };

__device__ inline Draw2 draw2(uint64_t seed, uint32_t w0, uint32_t step, uint32_t tag, uint32_t sub) {
    uint32_t c[4] = {w0, step, tag, sub};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    return {u52(c[0], c[1]), u52(c[2], c[3])};
}

__device__ inline bool inside_tip(const Grid& g, double X, double Y, double Z) {
    double dx = X - g.xc, dy = Y - g.yc;
    double rho2 = dx * dx + dy * dy;
    if (Z < 0.0) return false;
    if (Z <= g.zc) return rho2 <= g.R * g.R;
    double dz = Z - g.zc;
    return rho2 + dz * dz <= g.R * g.R;
}

// 0 inside the vacuum region, else the boundary a particle left through:
// 1 cathode plane, 2 anode plane, 3 lateral faces (also non-finite), 4 tip.
__device__ inline int boundary_code(const Grid& g, double X, double Y, double Z) {
    if (Z <= 0.0) return 1;
    if (Z >= (double)(g.nz - 1)) return 2;
    bool in = (X >= 0.0) && (X < (double)(g.nx - 1)) && (Y >= 0.0) && (Y < (double)(g.ny - 1)) &&
              (Z > 0.0) && (Z < (double)(g.nz - 1));
    if (!in) return 3;
    if (inside_tip(g, X, Y, Z)) return 4;
    return 0;
}

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// CIC weight of one axis quantized to 2^-bits, rounded half up (exact).
__device__ inline int64_t quantize(double f, int bits) {
    double t = ldexp(f, bits);
    double fl = floor(t);
    int64_t q = (int64_t)fl;
    if (t - fl >= 0.5) q += 1;
    return q;
}

__device__ inline int lane_id() { return __lane_id(); }

// Remap a block index so that consecutive chunks of the index space land on
// one XCD (blocks are dispatched round-robin over the 8 XCDs).
__device__ inline int64_t xcd_block(int64_t b, int64_t G) {
    int64_t per = G / 8, rem = G % 8;
    int64_t x = b % 8, t = b / 8;
    return x * per + (x < rem ? x : rem) + t;
}

// z-marching tiles for stencils on a node grid: blocks of 64 x 4 threads over
// (x, y) (block index remapped so that consecutive tiles share an XCD), each
// thread walking kc consecutive planes of one (x, y) column. Values of the
// planes below and above are carried in registers, so each step reads one new
// plane value per array; in-plane neighbours are L1/L2 hits.
struct ZMarch {
    int i, j, k0, k1;
    bool col;  // the column exists (the last x / y tiles may be partial)
};

__device__ inline ZMarch zmarch(int nx, int ny, int nz, int kc) {
    int ntx = (nx + 63) >> 6, nty = (ny + 3) >> 2;
    int64_t b = xcd_block(blockIdx.x, gridDim.x);
    int bx = (int)(b % ntx);
    int64_t r = b / ntx;
    int by = (int)(r % nty), bz = (int)(r / nty);
    ZMarch z;
    z.i = bx * 64 + (int)(threadIdx.x & 63);
    z.j = by * 4 + (int)(threadIdx.x >> 6);
    z.k0 = bz * kc;
    z.k1 = z.k0 + kc < nz ? z.k0 + kc : nz;
    z.col = z.i < nx && z.j < ny;
    return z;
}

// Grid of a z-marching launch of about `target` blocks (at most
// kMaxStencilBlocks where the grid allows); kc is rounded up to a multiple
// of `align`.
constexpr int kMaxStencilBlocks = 4096;
inline unsigned zmarch_grid(int nx, int ny, int nz, int target, int align, int* kc) {
    int64_t cols = (int64_t)((nx + 63) / 64) * ((ny + 3) / 4);
    int64_t k = (nz * cols + target - 1) / target;
    if (k < 1) k = 1;
    k = (k + align - 1) / align * align;
    while (k < nz && cols * ((nz + k - 1) / k) > kMaxStencilBlocks) k += align;  // partial-sum slots
    *kc = (int)k;
    return (unsigned)(cols * ((nz + k - 1) / k));
}

// Node coordinates along a strided walk n, n + step, n + 2 step, ... without
// divisions: the step is decomposed once in base (ny, nx) and carried.
struct NodeWalk {
    int i, j, k;
    int si, sj, sk, nx, ny;
    __device__ NodeWalk(int64_t n, int step, int nx_, int ny_) : nx(nx_), ny(ny_) {
        uint32_t n32 = (uint32_t)n, q = n32 / (uint32_t)nx;
        i = (int)(n32 - q * (uint32_t)nx);
        k = (int)(q / (uint32_t)ny);
        j = (int)(q - (uint32_t)k * (uint32_t)ny);
        si = step % nx;
        sj = (step / nx) % ny;
        sk = step / (nx * ny);
    }
    __device__ void advance() {
        i += si;
        int c = i >= nx;
        i -= c * nx;
        j += sj + c;
        int c2 = j >= ny;
        j -= c2 * ny;
        k += sk + c2;
    }
};

// Append from the active lanes with pred set: one atomic per wavefront,
// slots in lane order. Every active lane of the wavefront must call it.
__device__ inline unsigned long long wave_append(unsigned long long* ctr, bool pred) {
    uint64_t mask = __ballot(pred);
    if (mask == 0) return 0ull;
    int lane = __lane_id();
    int leader = __ffsll((unsigned long long)mask) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(ctr, (unsigned long long)__popcll(mask));
    base = __shfl(base, leader, 64);
    uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    return base + (unsigned long long)__popcll(mask & lt);
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block-wide sum in a fixed order (deterministic): wave sums then the first
// wave adds the wave results in index order.
template <typename T>
__device__ inline T block_sum(T v, T* sh) {
    v = wave_sum(v);
    int w = threadIdx.x / 64, l = threadIdx.x % 64;
    if (l == 0) sh[w] = v;
    __syncthreads();
    T r = T(0);
    if (threadIdx.x == 0) {
        for (int i = 0; i < (int)(blockDim.x + 63) / 64; ++i) r += sh[i];
    }
    __syncthreads();
    return r;  // valid in thread 0
}

// Sum of nparts (>= 1) per-block partials in a fixed order, returned to every
// thread of the block: each thread adds up to 8 strided values per round with
// the loads issued together (indices clamped, tail masked by a product), then
// a block reduction. Uses kBlock / 64 + 1 doubles of shared memory.
__device__ inline double sum_partials_n(const double* __restrict__ part, int nparts) {
    __shared__ double sh[kBlock / 64];
    __shared__ double res;
    double v = 0.0;
    for (int base = 0; base < nparts; base += 8 * (int)blockDim.x) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            int idx = base + u * (int)blockDim.x + (int)threadIdx.x;
            t[u] = part[idx < nparts ? idx : nparts - 1] * (double)(idx < nparts);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) v += t[u];
    }
    double tot = block_sum(v, sh);
    if (threadIdx.x == 0) res = tot;
    __syncthreads();
    return res;
}

}  // namespace pic

// Emission patches: fn_rings rings on the spherical cap, then one ring per
// spacing of the cylinder's height, each ring cut into fn_az sectors; the
// counts are taken by blocks of kInjCountBlock patches.
constexpr int kInjCountBlock = 256;
inline int64_t fn_patches(const pic_config* cfg) {
    if (cfg->fn_rings <= 0) return 0;
    const double zc = cfg->tip_h / cfg->h - cfg->tip_r / cfg->h;
    return ((int64_t)cfg->fn_rings + (int64_t)std::ceil(zc)) * cfg->fn_az;
}

// ---------------------------------------------------------------------------
// The context (host side).
struct pic_ctx {
    pic_config cfg;
    pic_buffers buf;
    hipStream_t stream;
    pic::Grid g;
    double V0 = 0.0, F1 = 0.0;
    double kq[3];                 // kick per step in grid units per V/m
    double adk_c = 0.0, adk_n = 0.0, fi_thr = 0.0, ebsi = 0.0;
    std::vector<double> nu_tab;   // host copy of the collision-rate bounds (2 x xs_n), uploaded after the tables
    int64_t npatch = 0;
    int64_t id_cap = 0, bm_words = 0;
    // scratch carve
    pic::DevState* st = nullptr;
    double* xs = nullptr;         // 3 * xs_n
    uint32_t* off = nullptr;      // nkeys + 1
    uint32_t* key[3] = {};
    uint2* bins = nullptr;        // sum cap: {species << 30 | slot, id} in cell order
    uint32_t* big = nullptr;      // big-cell list (nkeys)
    uint32_t* mcc_list = nullptr;   // small cells for the full collision pass (nkeys)
    uint32_t* mcc_count = nullptr;  // cells per scanning wavefront (4 x 8192)
    uint32_t* mcc_dense = nullptr;  // the listed cells, compacted (nkeys)
    uint32_t* fi_list = nullptr;  // cap neutral
    uint32_t* push_part = nullptr;  // per-block partials of the push kernels (8192 x 8)
    uint32_t* inj_cnt = nullptr;    // emission count of each patch (npatch)
    double* inj_part = nullptr;     // per-block expected counts and clamped patches of the emission
    uint32_t* nflag = nullptr;    // cap neutral: step+1 if the neutral had an event
    uint32_t* prod_list = nullptr;
    int32_t* prod_ev = nullptr;
    double* prod_ve = nullptr;    // 3 * cap neutral
    uint32_t* bitmap[2] = {};
    uint32_t* bm_prefix[2] = {};
    pic_event* ev = nullptr;
    int64_t ev_cap = 0;
    uint32_t* scan_blocks = nullptr;
    int64_t scan_blocks_n = 0;
    uint32_t* dyn = nullptr;      // small device-side counts (scan lengths and totals)
    uint32_t** id_ptrs = nullptr; // device copy of the three id array pointers
    uint32_t* bin_hist = nullptr;   // binning: [chunk][group] counts
    uint32_t* bin_segtot = nullptr; // [segment][group] totals
    uint32_t* bin_gbase = nullptr;  // [group + 1] first bins
    uint4* bin_stage = nullptr;     // elements in group order (sum cap)
    int bin_ng = 0, bin_gshift = 9; // groups, log2 of the cells per group
    uint32_t* rank_flag = nullptr;
    uint32_t* rank = nullptr;     // reorder destination ranks (per bin entry)
    void* tmp = nullptr;          // reorder staging: 6 arrays of tmp_cap elements + ids
    int64_t tmp_cap = 0;
    double* mom_out = nullptr;
    double *cg_r = nullptr, *cg_p0 = nullptr, *cg_p1 = nullptr, *cg_q = nullptr;
    double* partials = nullptr;
    int64_t partials_n = 0;
    void* mg = nullptr;           // multigrid work memory
    void* mg_host = nullptr;      // multigrid hierarchy (host description)
    void* mixed = nullptr;        // mixed-precision vectors
    struct unet* learned = nullptr;  // network of PIC_GUESS_LEARNED
    // captured pair of preconditioned CG iterations (built at the first
    // unprofiled multigrid solve)
    hipStream_t cap_stream = nullptr;
    // a step's collisions run on side_stream, concurrently with its Poisson
    // solve (which needs only the deposit): ev_dep orders them after the
    // deposit, ev_col orders the rest of the step after them
    hipStream_t side_stream = nullptr;
    hipEvent_t ev_dep = nullptr, ev_col = nullptr;
    hipGraph_t pcg_graph = nullptr, mix_graph = nullptr;
    hipGraphExec_t pcg_exec = nullptr, mix_exec = nullptr;
    int last_iters[3] = {0, 0, 0};   // iterations of the last solve per solver (first launch chunk)
    int learn_smooth = 0;            // binomial filter passes on its output
    int learn_project = 1;           // weight the network output by the energy-norm projection
    int learn_fallback = 1;          // judge the learned guess against V0 phi1 before each solve
    void* static_work = nullptr;     // this device's copy of the static work array (pic_inject_noalloc)
    double* push_dpart = nullptr;    // per-block FP64 partials of the push kernels (8192 x 4)
    // superparticle weights (cfg.weighted only)
    uint32_t* fi_cnt = nullptr;      // cap neutral: field-ionized units of a candidate neutral
    uint32_t* prod_c = nullptr;      // cap neutral: ionized units of a neutral with a product
    uint32_t* split_list[3] = {};    // per species: parent slots of the split-offs of the phase
    uint32_t* split_c[3] = {};       // per species and slot: units split off
    double* split_v[3] = {};         // per species and slot: velocity of the split-off (3 values)
    uint32_t* split_bm[3] = {};      // per species: split-off parents as a bitmap over ids
    uint32_t* split_pf[3] = {};      // their word prefix counts
    // recombination (cfg.same_species & 4 only)
    uint32_t* rec_list = nullptr;    // cap ion: slots of the recombined ions of the phase
    double* rec_v = nullptr;         // cap ion: velocity of the atom (3 values)
    uint32_t* rec_bm = nullptr;      // recombined ions as a bitmap over ids
    uint32_t* rec_pf = nullptr;      // its word prefix counts
    bool circuit = false;            // cfg.circuit_R > 0: the anode follows the RC circuit
    double evap_flux = 0.0;          // Clausius-Clapeyron flux at cfg.surface_T [1/(m^2 s)]
    double evap_vsig = 0.0;          // sqrt(k_B T / m) dt / h
    double* phi_prev = nullptr;      // potential of the previous step solve (extrapolated guess)
    int phi_hist = 0;                // consecutive step solves whose potential phi_prev / phi hold
    // host state
    pic::DevState* host_st = nullptr;  // pinned mirror
    int64_t step = 0;
    int bins_valid = 0, need_sort = 0;
    int64_t collide_count = 0;
    int failed = 0;
    std::string err;
    pic_solve_info last_solve{};
    int64_t cg_iters_total = 0;
    // profiling: pairs of events per timed interval
    int prof = 0;
    int push_all_handle = -1;
    hipEvent_t* evpool = nullptr;
    int ev_n = 0, ev_max = 0;
    int* ev_slot = nullptr;
    double t_ms[PIC_NTIMERS] = {};
    int64_t t_cnt[PIC_NTIMERS] = {};
};

namespace pic {
// the collide phase of this step merges superparticles
inline bool merge_step(const pic_ctx* c) {
    return c->cfg.merge_every > 0 && c->step % c->cfg.merge_every == 0;
}
// target block count of the z-marching solver kernels
inline int stencil_target(const pic_ctx* c) { return c->cfg.stencil_blocks ? c->cfg.stencil_blocks : 1024; }
size_t scratch_layout(pic_ctx* c, const pic_config* cfg, const int64_t cap[3], char* base);
hipError_t launch_node_types(pic_ctx* c);
hipError_t launch_field(pic_ctx* c, const double* phi, void* field);
// step-solve guess: phi <- 2 phi - phi_prev when apply; phi_prev <- phi
hipError_t extrapolate_phi(pic_ctx* c, bool apply);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
int cg_solve(pic_ctx* c, double* phi, double V0, const int64_t* rho, int guess, double rtol, int maxit,
             pic_solve_info* info);
int mg_setup(pic_ctx* c);
int mgcg_solve(pic_ctx* c, double* phi, double V0, const int64_t* rho, int guess, double rtol, int maxit,
               pic_solve_info* info);
int mixed_solve(pic_ctx* c, double* phi, double V0, const int64_t* rho, int guess, double rtol, int maxit,
                pic_solve_info* info);
size_t mg_bytes(const pic_config* cfg);
// z = V-cycle(b0) (FP32 z); b0 is the CG residual of the finest level
template <typename TB>
float* mg_vcycle(pic_ctx* c, const TB* b0, double* part_rr, double* part_bb, double* part_rz, int cg_blocks, int* n_rz,
                 bool timed);
void mg_free(pic_ctx* c);
hipError_t scan_u32(pic_ctx* c, const uint32_t* in, uint32_t* out, int64_t n_max, const uint32_t* nd,
                    uint32_t* total, bool zero_in, bool popcount);
hipError_t particles_phase(pic_ctx* c, bool move);
hipError_t collide_phase(pic_ctx* c, bool record);
hipError_t cell_bins(pic_ctx* c);
hipError_t inject_phase(pic_ctx* c);
// the emission with its per-patch counts and per-block sums in cnt and part
hipError_t inject_phase_in(pic_ctx* c, uint32_t* cnt, double* part);
// bytes of work memory of the surface injection (counts, block sums and, for
// the weights of evaporated neutrals, a {weight, atoms} pair per patch)
inline size_t inject_work_bytes(int64_t npatch) {
    const int64_t nb = (npatch + kInjCountBlock - 1) / kInjCountBlock;
    return (((size_t)npatch * 4 + 255) & ~(size_t)255) + (size_t)nb * 16 + (size_t)npatch * 8;
}
hipError_t load_particles(pic_ctx* c, const pic_particles* src);
hipError_t moments_phase(pic_ctx* c, double* out_dev);
hipError_t apex_interp(pic_ctx* c, const double* phi, double X, double Y, double Z, double* out_dev);
// phi = V0 phi1 (with_net = false) or V0 phi1 + network charge response
int guess_phi(pic_ctx* c, bool with_net);
// profiling: tic returns a handle for toc (or -1 when profiling is off)
int tic(pic_ctx* c, int slot);
void toc(pic_ctx* c, int h);
void flush_timers(pic_ctx* c);
}  // namespace pic
