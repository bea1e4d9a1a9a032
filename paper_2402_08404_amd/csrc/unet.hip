// unet.hip -- the learned warm start: a 3D U-Net mapping the normalized node
// charge to a potential guess, with forward, backward and Adam on the GPU.
//
// Convolutions are implicit GEMMs on the bf16 matrix cores
// (v_mfma_f32_16x16x32_bf16, fp32 accumulation): rows are output voxels,
// columns output channels, the reduction runs over (tap, input channel).
// Activations are bf16, channels last ([voxel][channel]); master weights,
// gradients and Adam moments are fp32. Gradients of activations are kept in
// fp32 and rounded to bf16 (with the ReLU mask applied) where a GEMM reads them.
//
// Architecture (4 levels, 16-32-64-128 channels): two 3x3x3 conv + ReLU per
// level, 2x2x2 stride-2 conv + ReLU down, 2x2x2 stride-2 transposed conv up,
// skip connections by channel concatenation, 1x1x1 linear head.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "pic_internal.hpp"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16_t;  // storage type of one bf16

namespace unet_impl {

constexpr int kModeSame3 = 0, kModeDown2 = 1, kModeUp2 = 2;

__device__ inline bf16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return (bf16_t)(u >> 16);  // inf / nan
    u += 0x7FFFu + ((u >> 16) & 1u);                                  // round to nearest even
    return (bf16_t)(u >> 16);
}
__device__ inline float bf2f(bf16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

struct Geo {
    int B, D, H, W;  // grid of the GEMM rows (output voxels, or coarse voxels for up)
    int iD, iH, iW;  // grid of the input tensor(s)
};

// ---------------------------------------------------------------------------
// Forward-type convolution (also used for input gradients).
// out[v][co] = act(bias[co] + sum_k A(v, k) W[co][k]),  k = tap * Cin + ci.
// mode Same3: 27 taps, input voxel v + offset(tap) (zero outside the sample);
//   flip: tap t reads offset(26 - t) (transposed stencil for input gradients).
// mode Down2: 8 taps, input voxel 2 v + offset(tap) on the finer input grid.
// mode Up2: rows are coarse voxels vc, one tap, output voxel 2 vc + par.
struct ConvArgs {
    const bf16_t* a;    // input A, channels ca
    const bf16_t* b;    // input B (concatenated after A), channels cb
    const bf16_t* w;    // [N][Kpad]
    const float* bias;  // [N] or null
    bf16_t* out;        // bf16 output [vox][N] or null
    float* out32;       // fp32 output [vox][N] or null
    int accumulate;     // out32 += result
    int ca, cb, N, K, Kpad, mode, relu, flip, par;
    Geo g;
};

// (x, y, z, sample) of row v, in 32-bit arithmetic (every tensor of the
// network holds fewer than 2^31 voxels)
__device__ inline void row_coords(const Geo& g, int64_t v, int& x, int& y, int& z, int& bsm) {
    const uint32_t u = (uint32_t)v, W = (uint32_t)g.W, H = (uint32_t)g.H, D = (uint32_t)g.D;
    const uint32_t q = u / W, q2 = q / H, q3 = q2 / D;
    x = (int)(u - q * W);
    y = (int)(q - q2 * H);
    z = (int)(q2 - q3 * D);
    bsm = (int)q3;
}

__device__ inline int src_voxel(const ConvArgs& p, int64_t v, int tap, bool& ok) {
    const Geo& g = p.g;
    int x, y, z, bsm;
    row_coords(g, v, x, y, z, bsm);
    int sx, sy, sz;
    if (p.mode == kModeSame3) {
        int t = p.flip ? 26 - tap : tap;
        sx = x + (t % 3) - 1;
        sy = y + ((t / 3) % 3) - 1;
        sz = z + (t / 9) - 1;
    } else if (p.mode == kModeDown2) {
        sx = 2 * x + (tap & 1);
        sy = 2 * y + ((tap >> 1) & 1);
        sz = 2 * z + ((tap >> 2) & 1);
    } else {
        sx = x;
        sy = y;
        sz = z;
    }
    ok = sx >= 0 && sx < g.iW && sy >= 0 && sy < g.iH && sz >= 0 && sz < g.iD;
    return (int)((((int64_t)bsm * g.iD + sz) * g.iH + sy) * g.iW + sx);
}

__device__ inline int64_t out_voxel(const ConvArgs& p, int64_t v) {
    if (p.mode != kModeUp2) return v;
    const Geo& g = p.g;
    int x, y, z, bsm;
    row_coords(g, v, x, y, z, bsm);
    int X = 2 * x + (p.par & 1), Y = 2 * y + ((p.par >> 1) & 1), Z = 2 * z + ((p.par >> 2) & 1);
    return (((int64_t)bsm * (2 * g.D) + Z) * (2 * g.H) + Y) * (2 * g.W) + X;
}

template <int NB>
__global__ __launch_bounds__(256) void k_conv(ConvArgs p) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t M = (int64_t)p.g.B * p.g.D * p.g.H * p.g.W;
    const int64_t row0 = (int64_t)blockIdx.x * 64 + wave * 16;
    const int64_t v = row0 + (lane & 15);
    const bool vrow = v < M;
    const int cin = p.ca + p.cb;
    f32x4 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = (f32x4){0.f, 0.f, 0.f, 0.f};
    const int kg = 8 * (lane >> 4);
    // the row's voxel coordinates, once (not per reduction step)
    const Geo& g = p.g;
    int x = 0, y = 0, z = 0, bsm = 0;
    {
        int64_t r = vrow ? v : 0;
        x = (int)(r % g.W);
        r /= g.W;
        y = (int)(r % g.H);
        r /= g.H;
        z = (int)(r % g.D);
        bsm = (int)(r / g.D);
    }
    for (int kc = 0; kc < p.Kpad; kc += 32) {
        int k0 = kc + kg;
        bf16x8 av;
        uint4 raw = make_uint4(0, 0, 0, 0);
        if (vrow && k0 < p.K) {
            const int tap = k0 / cin, ci = k0 - tap * cin;
            int sx = x, sy = y, sz = z;  // kModeUp2: the row's own voxel
            if (p.mode == kModeSame3) {
                const int t = p.flip ? 26 - tap : tap;
                sx += t % 3 - 1;
                sy += (t / 3) % 3 - 1;
                sz += t / 9 - 1;
            } else if (p.mode == kModeDown2) {
                sx = 2 * x + (tap & 1);
                sy = 2 * y + ((tap >> 1) & 1);
                sz = 2 * z + ((tap >> 2) & 1);
            }
            if (sx >= 0 && sx < g.iW && sy >= 0 && sy < g.iH && sz >= 0 && sz < g.iD) {
                const int64_t sv = (((int64_t)bsm * g.iD + sz) * g.iH + sy) * g.iW + sx;
                const bf16_t* src = ci < p.ca ? p.a + sv * p.ca + ci : p.b + sv * p.cb + (ci - p.ca);
                raw = *(const uint4*)src;
            }
        }
        av = *(bf16x8*)&raw;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const bf16_t* wp = p.w + (int64_t)(nb * 16 + (lane & 15)) * p.Kpad + k0;
            uint4 wr = *(const uint4*)wp;
            bf16x8 bv = *(bf16x8*)&wr;
            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[nb], 0, 0, 0);
        }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        int co = nb * 16 + (lane & 15);
        float bias = p.bias ? p.bias[co] : 0.f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int64_t r = row0 + 4 * (lane >> 4) + j;
            if (r >= M) continue;
            float val = acc[nb][j] + bias;
            if (p.relu) val = val > 0.f ? val : 0.f;
            int64_t o = out_voxel(p, r);
            if (p.out) p.out[o * p.N + co] = f2bf(val);
            if (p.out32) {
                float* q = p.out32 + o * p.N + co;
                *q = p.accumulate ? *q + val : val;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Up convolution (forward), all eight parities in one launch: each wave's 16
// coarse voxels are read once (their KS x 32 input channels kept in
// registers) and multiplied by the eight parities' weight slices in turn
// (slice par at w + par N Kpad), each writing its fine voxels 2 v + par.
template <int NB, int KS>
__global__ __launch_bounds__(256) void k_up2_all(ConvArgs p) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const Geo& g = p.g;
    const int64_t M = (int64_t)g.B * g.D * g.H * g.W;
    const int64_t row0 = (int64_t)blockIdx.x * 64 + wave * 16;
    const int64_t v = row0 + (lane & 15);
    const int kg = 8 * (lane >> 4);
    bf16x8 av[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int ci = 32 * ks + kg;
        uint4 raw = make_uint4(0, 0, 0, 0);
        if (v < M) raw = ci < p.ca ? *(const uint4*)(p.a + v * p.ca + ci) : *(const uint4*)(p.b + v * p.cb + (ci - p.ca));
        av[ks] = *(const bf16x8*)&raw;
    }
    // the coarse coordinates of the lane's four output rows
    int cx[4], cy[4], cz[4], cb[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        int64_t r = row0 + 4 * (lane >> 4) + j;
        cx[j] = (int)(r % g.W);
        r /= g.W;
        cy[j] = (int)(r % g.H);
        r /= g.H;
        cz[j] = (int)(r % g.D);
        cb[j] = (int)(r / g.D);
    }
    for (int par = 0; par < 8; ++par) {
        const bf16_t* w = p.w + (int64_t)par * p.N * p.Kpad;
        f32x4 acc[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const uint4 wr = *(const uint4*)(w + (int64_t)(nb * 16 + (lane & 15)) * p.Kpad + 32 * ks + kg);
                acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[ks], *(const bf16x8*)&wr, acc[nb], 0, 0, 0);
            }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int co = nb * 16 + (lane & 15);
            const float bias = p.bias ? p.bias[co] : 0.f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (row0 + 4 * (lane >> 4) + j >= M) continue;
                float val = acc[nb][j] + bias;
                if (p.relu) val = val > 0.f ? val : 0.f;
                const int X = 2 * cx[j] + (par & 1), Y = 2 * cy[j] + ((par >> 1) & 1), Z = 2 * cz[j] + (par >> 2);
                const int64_t o = (((int64_t)cb[j] * (2 * g.D) + Z) * (2 * g.H) + Y) * (2 * g.W) + X;
                p.out[o * p.N + co] = f2bf(val);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// 3x3x3 convolution (forward, or input gradient with flip) with the input
// tile in LDS. A block owns an output tile of 32 x 4 x 2 voxels (x, y, z):
// 256 GEMM rows = 16 M-tiles of 16 consecutive x voxels, wave w taking
// M-tiles w, w+4, w+8, w+12, and all N output channels. The input channels
// are taken in chunks of CH = min(cin, 32): for each chunk the tile with a
// one-voxel halo (34 x 6 x 4 voxels x CH channels, bf16, zero outside the
// volume) is staged in LDS, then all 27 taps of the chunk are reduced; an A
// fragment is one 16-byte LDS read (8 channels of one voxel at the tap's
// offset), a B fragment one 16-byte read of the packed weights (k = tap cin +
// channel), shared by the wave's four M-tiles.
constexpr int kTX = 32, kTY = 4, kTZ = 2;
constexpr int kHX = kTX + 2, kHY = kTY + 2, kHZ = kTZ + 2;
constexpr int kHalo = kHX * kHY * kHZ;  // 816 voxels
constexpr int kChunk = 32;               // input channels per staged chunk

__host__ __device__ inline int conv3_tiles(const Geo& g) {
    return ((g.W + kTX - 1) / kTX) * ((g.H + kTY - 1) / kTY) * ((g.D + kTZ - 1) / kTZ) * g.B;
}

// The chunk width CH (8, 16 or 32) is fixed at compile time: a 32-wide
// reduction step covers 32 / CH taps, so a lane's tap and channel follow
// from shifts and the tap's halo offset from two multiply-shifts; the loads
// of a chunk's halo tile are all issued before it is written to LDS, and the
// B fragments of the next step are loaded while the current step's MFMAs
// run. The LDS tile holds CH channels (13, 26 or 52 KB). On the small
// levels the output channels are split over blockIdx.y (NB x 16 a block), so
// that the grid fills the GPU.
template <int NB, int CH>
__global__ __launch_bounds__(256) void k_conv3_ch(ConvArgs p) {
    static_assert(CH == 8 || CH == 16 || CH == 32, "chunk width");
    __shared__ __align__(16) bf16_t tile[kHalo * CH];
    const int cin = p.ca + p.cb;
    const Geo& g = p.g;
    const int ntx = (g.W + kTX - 1) / kTX, nty = (g.H + kTY - 1) / kTY, ntz = (g.D + kTZ - 1) / kTZ;
    int bid = (int)pic::xcd_block(blockIdx.x, gridDim.x);  // neighbouring tiles (their halos) on one XCD
    const int tx = bid % ntx;
    bid /= ntx;
    const int ty = bid % nty;
    bid /= nty;
    const int tz = bid % ntz;
    const int bsm = bid / ntz;
    const int x0 = tx * kTX, y0 = ty * kTY, z0 = tz * kTZ;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, kg = 8 * (lane >> 4);
    const int n0 = (int)blockIdx.y * NB * 16;  // the block's first output channel (channel groups along y)
    constexpr int kSteps = (27 * CH + 31) / 32;  // reduction steps of one chunk
    constexpr int kTapsPerStep = 32 / CH;
    // the halo voxel of each of the wave's four M-tiles at tap offset zero
    int base[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int m = wave + 4 * q;
        const int lx = 16 * (m & 1) + r16, ly = (m >> 1) & 3, lz = m >> 3;
        base[q] = ((lz + 1) * kHY + (ly + 1)) * kHX + (lx + 1);
    }
    // the lane's tap (valid or not), channel within the chunk and halo offset at step s
    auto lane_tap = [&](int s, int& tap, int& cc, int& off) {
        tap = s * kTapsPerStep + kg / CH;
        cc = kg % CH;
        const bool valid = tap < 27;  // past the last tap: a zero A fragment
        if (!valid) tap = 0;
        const int t = p.flip ? 26 - tap : tap;
        const int dz = (t * 57) >> 9, r = t - 9 * dz;  // t / 9 and t % 9 for t < 27
        const int dy = (r * 11) >> 5, dx = r - 3 * dy;  // r / 3 and r % 3 for r < 9
        off = ((dz - 1) * kHY + (dy - 1)) * kHX + (dx - 1);
        return valid;
    };
    f32x4 acc[4][NB];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[q][nb] = (f32x4){0.f, 0.f, 0.f, 0.f};
    constexpr int c8n = CH / 8;
    constexpr int kLoads = (kHalo * c8n + 255) / 256;  // 16-byte loads a thread per chunk
    for (int c0 = 0; c0 < cin; c0 += CH) {
        // every load of the chunk's halo tile is issued before the first LDS
        // write (the loop is unrolled into registers)
        uint4 stage[kLoads];
#pragma unroll
        for (int it = 0; it < kLoads; ++it) {
            const int e = (int)threadIdx.x + 256 * it;
            const int vox = e / c8n, c8 = (e - vox * c8n) * 8;
            const int hx = vox % kHX, hy = (vox / kHX) % kHY, hz = vox / (kHX * kHY);
            const int X = x0 + hx - 1, Y = y0 + hy - 1, Z = z0 + hz - 1;
            stage[it] = make_uint4(0, 0, 0, 0);
            if (e < kHalo * c8n && X >= 0 && X < g.W && Y >= 0 && Y < g.H && Z >= 0 && Z < g.D) {
                const int64_t sv = (((int64_t)bsm * g.D + Z) * g.H + Y) * g.W + X;
                const int ch = c0 + c8;
                stage[it] = ch < p.ca ? *(const uint4*)(p.a + sv * p.ca + ch)
                                      : *(const uint4*)(p.b + sv * p.cb + (ch - p.ca));
            }
        }
        if (c0) __syncthreads();  // the previous chunk's reads are done
#pragma unroll
        for (int it = 0; it < kLoads; ++it) {
            const int e = (int)threadIdx.x + 256 * it;
            if (e < kHalo * c8n) *(uint4*)(tile + e * 8) = stage[it];  // (vox * CH + c8) = 8 e
        }
        __syncthreads();
        auto load_b = [&](int s, bf16x8* bv) {
            int tap, cc, off;
            lane_tap(s, tap, cc, off);
            const int64_t kw = (int64_t)tap * cin + c0 + cc;  // column of the packed weights
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const uint4 wr = *(const uint4*)(p.w + (int64_t)(n0 + nb * 16 + r16) * p.Kpad + kw);
                bv[nb] = *(const bf16x8*)&wr;
            }
        };
        bf16x8 bcur[NB], bnext[NB];
        load_b(0, bcur);
        auto step = [&](int s) {
            if (s + 1 < kSteps) load_b(s + 1, bnext);
            int tap, cc, off;
            const bool valid = lane_tap(s, tap, cc, off);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint4 raw = make_uint4(0, 0, 0, 0);
                if (valid) raw = *(const uint4*)(tile + (base[q] + off) * CH + cc);
                const bf16x8 av = *(const bf16x8*)&raw;
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[q][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bcur[nb], acc[q][nb], 0, 0, 0);
            }
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) bcur[nb] = bnext[nb];
        };
        // (measured: the compiler's unrolling pays at 32 channels, a rolled
        // loop with its higher occupancy at 8 and 16)
        if constexpr (CH == 32) {
            for (int s = 0; s < kSteps; ++s) step(s);
        } else {
#pragma unroll 1
            for (int s = 0; s < kSteps; ++s) step(s);
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int m = wave + 4 * q;
        const int ly = (m >> 1) & 3, lz = m >> 3;
        const int Y = y0 + ly, Z = z0 + lz;
        if (Y >= g.H || Z >= g.D) continue;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int co = n0 + nb * 16 + r16;
            const float bias = p.bias ? p.bias[co] : 0.f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int X = x0 + 16 * (m & 1) + 4 * (lane >> 4) + j;
                if (X >= g.W) continue;
                float val = acc[q][nb][j] + bias;
                if (p.relu) val = val > 0.f ? val : 0.f;
                const int64_t o = (((int64_t)bsm * g.D + Z) * g.H + Y) * g.W + X;
                if (p.out) p.out[o * p.N + co] = f2bf(val);
                if (p.out32) {
                    float* dst = p.out32 + o * p.N + co;
                    *dst = p.accumulate ? *dst + val : val;
                }
            }
        }
    }
}

// Persistent form for the large single-chunk layers (cin = CH = 8 or 16):
// a block takes a contiguous range of tiles, keeps the layer's weights in LDS
// (loaded once), and loads the next tile's halo into registers while the
// current tile's MFMAs run, so the staging latency overlaps the compute (the
// compute reads only LDS, so no wait for a global load sits inside it).
template <int NB, int CH>
__global__ __launch_bounds__(256) void k_conv3_ps(ConvArgs p) {
    static_assert(CH == 8 || CH == 16, "single-chunk widths");
    constexpr int kSpan = 27 * CH;                // reduction length (one chunk)
    constexpr int kSteps = (kSpan + 31) / 32;
    constexpr int kTapsPerStep = 32 / CH;
    constexpr int kPitch = kSteps * 32;           // LDS row of the weights (zero-padded)
    __shared__ __align__(16) bf16_t tile[kHalo * CH];
    __shared__ __align__(16) bf16_t wts[NB * 16 * kPitch];
    const Geo& g = p.g;
    const int ntx = (g.W + kTX - 1) / kTX, nty = (g.H + kTY - 1) / kTY, ntz = (g.D + kTZ - 1) / kTZ;
    const int ntiles = ntx * nty * ntz * g.B;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, kg = 8 * (lane >> 4);
    const int n0 = (int)blockIdx.y * NB * 16;
    // the weights of the block's output channels, once
    for (int e = threadIdx.x; e < NB * 16 * (kPitch / 8); e += 256) {
        const int row = e / (kPitch / 8), k8 = (e - row * (kPitch / 8)) * 8;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (k8 < kSpan) v = *(const uint4*)(p.w + (int64_t)(n0 + row) * p.Kpad + k8);
        *(uint4*)(wts + row * kPitch + k8) = v;
    }
    int base[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int m = wave + 4 * q;
        const int lx = 16 * (m & 1) + r16, ly = (m >> 1) & 3, lz = m >> 3;
        base[q] = ((lz + 1) * kHY + (ly + 1)) * kHX + (lx + 1);
    }
    constexpr int c8n = CH / 8;
    constexpr int kLoads = (kHalo * c8n + 255) / 256;
    auto coords = [&](int t, int& x0, int& y0, int& z0, int& bsm) {
        const int tx = t % ntx;
        t /= ntx;
        const int ty = t % nty;
        t /= nty;
        const int tz = t % ntz;
        bsm = t / ntz;
        x0 = tx * kTX;
        y0 = ty * kTY;
        z0 = tz * kTZ;
    };
    auto fetch = [&](int t, uint4* st) {
        int x0, y0, z0, bsm;
        coords(t, x0, y0, z0, bsm);
#pragma unroll
        for (int it = 0; it < kLoads; ++it) {
            const int e = (int)threadIdx.x + 256 * it;
            const int vox = e / c8n, c8 = (e - vox * c8n) * 8;
            const int hx = vox % kHX, hy = (vox / kHX) % kHY, hz = vox / (kHX * kHY);
            const int X = x0 + hx - 1, Y = y0 + hy - 1, Z = z0 + hz - 1;
            st[it] = make_uint4(0, 0, 0, 0);
            if (e < kHalo * c8n && X >= 0 && X < g.W && Y >= 0 && Y < g.H && Z >= 0 && Z < g.D) {
                const int64_t sv = (((int64_t)bsm * g.D + Z) * g.H + Y) * g.W + X;
                st[it] = c8 < p.ca ? *(const uint4*)(p.a + sv * p.ca + c8)
                                   : *(const uint4*)(p.b + sv * p.cb + (c8 - p.ca));
            }
        }
    };
    const int64_t lb = pic::xcd_block(blockIdx.x, gridDim.x);
    const int t0 = (int)(lb * ntiles / gridDim.x), t1 = (int)((lb + 1) * ntiles / gridDim.x);
    uint4 stage[kLoads];
    if (t0 < t1) fetch(t0, stage);
    for (int t = t0; t < t1; ++t) {
        __syncthreads();  // the previous tile's LDS reads are done (and the weights written)
#pragma unroll
        for (int it = 0; it < kLoads; ++it) {
            const int e = (int)threadIdx.x + 256 * it;
            if (e < kHalo * c8n) *(uint4*)(tile + e * 8) = stage[it];
        }
        __syncthreads();
        int x0, y0, z0, bsm;
        coords(t, x0, y0, z0, bsm);
        if (t + 1 < t1) fetch(t + 1, stage);  // in flight during this tile's MFMAs
        f32x4 acc[4][NB];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[q][nb] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
        for (int s = 0; s < kSteps; ++s) {
            int tap = s * kTapsPerStep + kg / CH;
            const int cc = kg % CH;
            const bool valid = tap < 27;
            if (!valid) tap = 0;
            const int tt = p.flip ? 26 - tap : tap;
            const int dz = (tt * 57) >> 9, r = tt - 9 * dz;
            const int dy = (r * 11) >> 5, dx = r - 3 * dy;
            const int off = ((dz - 1) * kHY + (dy - 1)) * kHX + (dx - 1);
            bf16x8 bv[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) bv[nb] = *(const bf16x8*)(wts + (nb * 16 + r16) * kPitch + 32 * s + kg);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint4 raw = make_uint4(0, 0, 0, 0);
                if (valid) raw = *(const uint4*)(tile + (base[q] + off) * CH + cc);
                const bf16x8 av = *(const bf16x8*)&raw;
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[q][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[nb], acc[q][nb], 0, 0, 0);
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int m = wave + 4 * q;
            const int ly = (m >> 1) & 3, lz = m >> 3;
            const int Y = y0 + ly, Z = z0 + lz;
            if (Y >= g.H || Z >= g.D) continue;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int co = n0 + nb * 16 + r16;
                const float bias = p.bias ? p.bias[co] : 0.f;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int X = x0 + 16 * (m & 1) + 4 * (lane >> 4) + j;
                    if (X >= g.W) continue;
                    float val = acc[q][nb][j] + bias;
                    if (p.relu) val = val > 0.f ? val : 0.f;
                    const int64_t o = (((int64_t)bsm * g.D + Z) * g.H + Y) * g.W + X;
                    if (p.out) p.out[o * p.N + co] = f2bf(val);
                    if (p.out32) {
                        float* dst = p.out32 + o * p.N + co;
                        *dst = p.accumulate ? *dst + val : val;
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Weight gradient: dW[tap][ci][co] = sum_v A(v, tap)[ci] G[v][co] over the
// GEMM rows v of the forward layer; split over row ranges, partials written
// per split and summed in a fixed order afterwards.
struct WgradArgs {
    const bf16_t* a;
    const bf16_t* b;
    const bf16_t* gr;   // G [rows][N] (output-voxel order of the forward)
    float* part;        // [nsplit][taps][cin][N]
    int ca, cb, N, taps, mode, par;
    int64_t rows_per_split;
    Geo g;
};

template <int MB, int NBW>
__global__ __launch_bounds__(256) void k_wgrad(WgradArgs p) {
    // block: one tap and one split; 4 waves share the (cin x N) tiles
    __shared__ __align__(16) bf16_t As[32][128 + 8];
    __shared__ __align__(16) bf16_t Gs[32][128 + 8];
    const int tap = blockIdx.x % p.taps;
    const int split = blockIdx.x / p.taps;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cin = p.ca + p.cb;
    const int64_t M = (int64_t)p.g.B * p.g.D * p.g.H * p.g.W;
    int64_t r0 = (int64_t)split * p.rows_per_split, r1 = r0 + p.rows_per_split;
    if (r1 > M) r1 = M;
    const int cin16 = (cin + 15) / 16 * 16;  // the 8-channel input is padded with zero columns
    const int mt = cin16 / 16, nt = p.N / 16;
    const int ntile = mt * nt;
    f32x4 acc[MB * NBW];
#pragma unroll
    for (int q = 0; q < MB * NBW; ++q) acc[q] = (f32x4){0.f, 0.f, 0.f, 0.f};
    ConvArgs cp;
    cp.mode = p.mode;
    cp.flip = 0;
    cp.par = p.par;
    cp.g = p.g;
    for (int64_t rb = r0; rb < r1; rb += 32) {
        // stage 32 rows of A (the tap's input voxels) and of G
        for (int e = threadIdx.x; e < 32 * (cin16 / 8); e += blockDim.x) {
            int rr = e / (cin16 / 8), c8 = (e % (cin16 / 8)) * 8;
            int64_t v = rb + rr;
            uint4 raw = make_uint4(0, 0, 0, 0);
            if (v < r1 && c8 < cin) {
                bool ok = true;
                int s = src_voxel(cp, v, tap, ok);
                if (ok) raw = c8 < p.ca ? *(const uint4*)(p.a + (int64_t)s * p.ca + c8)
                                        : *(const uint4*)(p.b + (int64_t)s * p.cb + (c8 - p.ca));
            }
            *(uint4*)&As[rr][c8] = raw;
        }
        for (int e = threadIdx.x; e < 32 * (p.N / 8); e += blockDim.x) {
            int rr = e / (p.N / 8), c8 = (e % (p.N / 8)) * 8;
            int64_t v = rb + rr;
            uint4 raw = make_uint4(0, 0, 0, 0);
            if (v < r1) {
                int64_t o = out_voxel(cp, v);
                raw = *(const uint4*)(p.gr + o * p.N + c8);
            }
            *(uint4*)&Gs[rr][c8] = raw;
        }
        __syncthreads();
        // C[ci][co] += A^T[ci][row] G[row][co]: K = 32 rows
        const int kg = 8 * (lane >> 4);
#pragma unroll
        for (int q = 0; q < MB * NBW; ++q) {
            int tile = wave + 4 * q;
            if (tile < ntile) {
                int mb = tile / nt, nb = tile % nt;
                bf16x8 av, bv;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    bf16_t x = As[kg + j][mb * 16 + (lane & 15)];
                    bf16_t y = Gs[kg + j][nb * 16 + (lane & 15)];
                    av[j] = *(__bf16*)&x;
                    bv[j] = *(__bf16*)&y;
                }
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[q], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < MB * NBW; ++q) {
        int tile = wave + 4 * q;
        if (tile < ntile) {
            int mb = tile / nt, nb = tile % nt;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                int ci = mb * 16 + 4 * (lane >> 4) + j, co = nb * 16 + (lane & 15);
                if (ci < cin) p.part[(((int64_t)split * p.taps + tap) * cin + ci) * p.N + co] = acc[q][j];
            }
        }
    }
}

// Weight gradient with larger staged chunks (R rows) and work for every
// wave: with at least four (ci, co) tiles the waves split the tiles; with
// fewer, each wave takes one 32-row step of every chunk (R = 128) and the four
// partial sums are added in wave order at the end. The next chunk's rows are
// loaded into registers while the current chunk is reduced.
template <int R>
__global__ __launch_bounds__(256) void k_wgrad2(WgradArgs p) {
    constexpr int LD = (R == 128 ? 64 : 128) + 8;  // LDS row pitch (channels + pad)
    constexpr int IT = (R * (LD - 8) / 8 + 255) / 256;  // staged items per thread and operand (max)
    __shared__ __align__(16) bf16_t As[R][LD];
    __shared__ __align__(16) bf16_t Gs[R][LD];
    const int tap = blockIdx.x % p.taps;
    const int split = blockIdx.x / p.taps;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cin = p.ca + p.cb;
    const int64_t M = (int64_t)p.g.B * p.g.D * p.g.H * p.g.W;
    int64_t r0 = (int64_t)split * p.rows_per_split, r1 = r0 + p.rows_per_split;
    if (r1 > M) r1 = M;
    const int cin16 = (cin + 15) / 16 * 16;  // the 8-channel input is padded with zero columns
    const int mt = cin16 / 16, nt = p.N / 16;
    const int ntile = mt * nt;
    const bool split_k = R == 128 && ntile < 4;  // the reduction scratch fits the R = 128 tile
    const int a8 = cin16 / 8, g8 = p.N / 8;
    ConvArgs cp;
    cp.mode = p.mode;
    cp.flip = 0;
    cp.par = p.par;
    cp.g = p.g;
    uint4 ra[IT], rg[IT];
    auto fetch = [&](int64_t rb) {
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int e = threadIdx.x + it * 256;
            uint4 va = make_uint4(0, 0, 0, 0), vg = make_uint4(0, 0, 0, 0);
            if (e < R * a8) {
                const int rr = e / a8, c8 = (e - rr * a8) * 8;
                const int64_t v = rb + rr;
                if (v < r1 && c8 < cin) {
                    bool ok = true;
                    const int sv = src_voxel(cp, v, tap, ok);
                    if (ok)
                        va = c8 < p.ca ? *(const uint4*)(p.a + (int64_t)sv * p.ca + c8)
                                       : *(const uint4*)(p.b + (int64_t)sv * p.cb + (c8 - p.ca));
                }
            }
            if (e < R * g8) {
                const int rr = e / g8, c8 = (e - rr * g8) * 8;
                const int64_t v = rb + rr;
                if (v < r1) vg = *(const uint4*)(p.gr + out_voxel(cp, v) * p.N + c8);
            }
            ra[it] = va;
            rg[it] = vg;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int e = threadIdx.x + it * 256;
            if (e < R * a8) {
                const int rr = e / a8, c8 = (e - rr * a8) * 8;
                *(uint4*)&As[rr][c8] = ra[it];
            }
            if (e < R * g8) {
                const int rr = e / g8, c8 = (e - rr * g8) * 8;
                *(uint4*)&Gs[rr][c8] = rg[it];
            }
        }
    };
    f32x4 acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = (f32x4){0.f, 0.f, 0.f, 0.f};
    const int kg = 8 * (lane >> 4);
    if (r0 < r1) fetch(r0);
    for (int64_t rb = r0; rb < r1; rb += R) {
        __syncthreads();  // the previous chunk's LDS reads are done
        store();
        __syncthreads();
        if (rb + R < r1) fetch(rb + R);
        for (int sub = split_k ? wave : 0; sub < R / 32; sub += split_k ? 4 : 1) {
            const int kr = 32 * sub + kg;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int tile = split_k ? q : wave + 4 * q;
                if (tile < ntile) {
                    const int mb = tile / nt, nb = tile % nt;
                    bf16x8 av, bv;
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        bf16_t x = As[kr + j][mb * 16 + (lane & 15)];
                        bf16_t y = Gs[kr + j][nb * 16 + (lane & 15)];
                        av[j] = *(__bf16*)&x;
                        bv[j] = *(__bf16*)&y;
                    }
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[q], 0, 0, 0);
                }
            }
        }
    }
    float* base = p.part + ((int64_t)split * p.taps + tap) * cin * p.N;
    if (split_k) {
        // partial sums of the four waves, added in wave order
        __syncthreads();
        float* red = (float*)&As[0][0];  // 4 waves x 3 tiles x 64 lanes x 4 values
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j) red[((wave * 3 + q) * 64 + lane) * 4 + j] = acc[q][j];
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                if (q >= ntile) break;
                const int mb = q / nt, nb = q % nt;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float v = 0.f;
                    for (int w = 0; w < 4; ++w) v += red[((w * 3 + q) * 64 + lane) * 4 + j];
                    const int ci = mb * 16 + 4 * (lane >> 4) + j, co = nb * 16 + (lane & 15);
                    if (ci < cin) base[(int64_t)ci * p.N + co] = v;
                }
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int tile = wave + 4 * q;
            if (tile < ntile) {
                const int mb = tile / nt, nb = tile % nt;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int ci = mb * 16 + 4 * (lane >> 4) + j, co = nb * 16 + (lane & 15);
                    if (ci < cin) base[(int64_t)ci * p.N + co] = acc[q][j];
                }
            }
        }
    }
}

// Weight gradient of a 3x3x3 convolution in one pass over the voxels for
// all 27 taps: a block takes a contiguous range of output tiles of
// 32 x 4 x 2 voxels in turn, stages the tile's input
// with its one-voxel halo (CH channels) and its output gradient (NT x 16
// channels) in LDS, and adds A(v + offset(tap))[ci] G(v)[co] over the tile's
// 256 voxels for every tap (wave w taking taps w, w + 4, ...), eight voxels
// of one x row per lane and reduction step. The input channels are taken CH
// at a time, chunk blockIdx.y. The block's sums go to
// part[block][tap][ci][co], summed over the blocks in a fixed order after.
template <int CH, int NT>
__global__ __launch_bounds__(256) void k_wgrad3(WgradArgs p) {
    static_assert(CH == 8 || CH == 16 || CH == 32, "input channels");
    constexpr int NC = NT * 16;
    constexpr int CT = (CH + 15) / 16;          // ci tiles (rows past CH are zero)
    constexpr int kTapsW = 7;                   // taps of a wave (at most)
    __shared__ __align__(16) bf16_t As[kHalo * CH];
    __shared__ __align__(16) bf16_t Gs[kTX * kTY * kTZ * NC];
    const Geo& g = p.g;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, kg = 8 * (lane >> 4);
    const int ntx = (g.W + kTX - 1) / kTX, nty = (g.H + kTY - 1) / kTY, ntz = (g.D + kTZ - 1) / kTZ;
    const int ntiles = ntx * nty * ntz * g.B;
    const int cin = p.ca + p.cb, c0 = (int)blockIdx.y * CH;  // all input channels; the block's first
    f32x4 acc[kTapsW][CT][NT];
#pragma unroll
    for (int i = 0; i < kTapsW; ++i)
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int n = 0; n < NT; ++n) acc[i][c][n] = (f32x4){0.f, 0.f, 0.f, 0.f};
    constexpr int c8a = CH / 8, c8g = NC / 8;
    constexpr int kLoadA = (kHalo * c8a + 255) / 256, kLoadG = (kTX * kTY * kTZ * c8g + 255) / 256;
    // the block's tiles: a contiguous range, the blocks of one XCD holding
    // neighbouring ranges (halos shared in its L2)
    const int64_t lb = pic::xcd_block(blockIdx.x, gridDim.x);
    const int t0 = (int)(lb * ntiles / gridDim.x), t1 = (int)((lb + 1) * ntiles / gridDim.x);
    for (int tile = t0; tile < t1; ++tile) {
        int bid = tile;
        const int tx = bid % ntx;
        bid /= ntx;
        const int ty = bid % nty;
        bid /= nty;
        const int tz = bid % ntz;
        const int bsm = bid / ntz;
        const int x0 = tx * kTX, y0 = ty * kTY, z0 = tz * kTZ;
        // every load of the tile issued before the first LDS write
        uint4 sa[kLoadA], sg[kLoadG];
#pragma unroll
        for (int it = 0; it < kLoadA; ++it) {
            const int e = (int)threadIdx.x + 256 * it;
            const int vox = e / c8a, c8 = (e - vox * c8a) * 8;
            const int hx = vox % kHX, hy = (vox / kHX) % kHY, hz = vox / (kHX * kHY);
            const int X = x0 + hx - 1, Y = y0 + hy - 1, Z = z0 + hz - 1;
            sa[it] = make_uint4(0, 0, 0, 0);
            if (e < kHalo * c8a && X >= 0 && X < g.W && Y >= 0 && Y < g.H && Z >= 0 && Z < g.D) {
                const int64_t sv = (((int64_t)bsm * g.D + Z) * g.H + Y) * g.W + X;
                const int ch = c0 + c8;
                sa[it] = ch < p.ca ? *(const uint4*)(p.a + sv * p.ca + ch)
                                   : *(const uint4*)(p.b + sv * p.cb + (ch - p.ca));
            }
        }
#pragma unroll
        for (int it = 0; it < kLoadG; ++it) {
            const int e = (int)threadIdx.x + 256 * it;
            const int vox = e / c8g, c8 = (e - vox * c8g) * 8;
            const int lx = vox % kTX, ly = (vox / kTX) % kTY, lz = vox / (kTX * kTY);
            const int X = x0 + lx, Y = y0 + ly, Z = z0 + lz;
            sg[it] = make_uint4(0, 0, 0, 0);
            if (e < kTX * kTY * kTZ * c8g && X < g.W && Y < g.H && Z < g.D) {
                const int64_t v = (((int64_t)bsm * g.D + Z) * g.H + Y) * g.W + X;
                sg[it] = *(const uint4*)(p.gr + v * NC + c8);
            }
        }
        __syncthreads();  // the previous tile's LDS reads are done
#pragma unroll
        for (int it = 0; it < kLoadA; ++it) {
            const int e = (int)threadIdx.x + 256 * it;
            if (e < kHalo * c8a) *(uint4*)(As + 8 * e) = sa[it];
        }
#pragma unroll
        for (int it = 0; it < kLoadG; ++it) {
            const int e = (int)threadIdx.x + 256 * it;
            if (e < kTX * kTY * kTZ * c8g) *(uint4*)(Gs + 8 * e) = sg[it];
        }
        __syncthreads();
        // reduction steps: the 8 x rows of the tile, 32 voxels each
        for (int row = 0; row < kTY * kTZ; ++row) {
            const int ly = row % kTY, lz = row / kTY;
            bf16x8 bv[NT];
#pragma unroll
            for (int n = 0; n < NT; ++n)
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const bf16_t y = Gs[(row * kTX + kg + j) * NC + n * 16 + r16];
                    bv[n][j] = *(const __bf16*)&y;
                }
            const int hrow = ((lz + 1) * kHY + (ly + 1)) * kHX + 1 + kg;  // halo voxel of x = kg, offset zero
#pragma unroll
            for (int i = 0; i < kTapsW; ++i) {
                const int t = wave + 4 * i;
                if (t >= 27) break;
                const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
                const int h0 = hrow + (dz * kHY + dy) * kHX + dx;
#pragma unroll
                for (int c = 0; c < CT; ++c) {
                    bf16x8 av;
                    const int ci = c * 16 + r16;
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const bf16_t x = ci < CH ? As[(h0 + j) * CH + ci] : (bf16_t)0;
                        av[j] = *(const __bf16*)&x;
                    }
#pragma unroll
                    for (int n = 0; n < NT; ++n)
                        acc[i][c][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[n], acc[i][c][n], 0, 0, 0);
                }
            }
        }
    }
    float* base = p.part + (int64_t)blockIdx.x * 27 * cin * NC;
#pragma unroll
    for (int i = 0; i < kTapsW; ++i) {
        const int t = wave + 4 * i;
        if (t >= 27) break;
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int n = 0; n < NT; ++n)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int ci = c * 16 + 4 * (lane >> 4) + j, co = n * 16 + r16;
                    if (ci < CH) base[((int64_t)t * cin + c0 + ci) * NC + co] = acc[i][c][n][j];
                }
    }
}

// gW[i] = sum over splits of part[s][i] (fixed order)
// (eight loads in flight, added in split order)
__global__ void k_sum_splits(const float* part, int nsplit, int64_t n, float* gw) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    int k = 0;
    for (; k + 8 <= nsplit; k += 8) {
        float t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = part[(int64_t)(k + u) * n + i];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += t[u];
    }
    for (; k < nsplit; ++k) s += part[(int64_t)k * n + i];
    gw[i] = s;
}

// gb[co] = sum over voxels of G[v][co]: per-block partial sums then a final
// pass in a fixed order.
__global__ void k_bias_partial(const float* g32, int64_t M, int N, float* part) {
    int co = threadIdx.x % N;
    int lanes = blockDim.x / N;
    int sub = threadIdx.x / N;
    float s = 0.f;
    int64_t per = (M + gridDim.x - 1) / gridDim.x;
    int64_t v0 = (int64_t)blockIdx.x * per, v1 = v0 + per < M ? v0 + per : M;
    for (int64_t v = v0 + sub; v < v1; v += lanes) s += g32[v * N + co];
    __shared__ float sh[256];
    sh[threadIdx.x] = s;
    __syncthreads();
    if (sub == 0) {
        float t = 0.f;
        for (int q = 0; q < lanes; ++q) t += sh[q * N + co];
        part[(int64_t)blockIdx.x * N + co] = t;
    }
}

// G (bf16) = g32 * (y > 0) for a ReLU layer, or g32 for a linear one; the
// fp32 gradient after the mask is kept for the bias gradient.
__global__ void k_mask(const float* g32, const bf16_t* y, int relu, int64_t n, bf16_t* G, float* gm32) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float v = g32[i];
    if (relu && !(bf2f(y[i]) > 0.f)) v = 0.f;
    G[i] = f2bf(v);
    gm32[i] = v;
}

// Input: normalized charge (fp32 [vox]) into a bf16 tensor of 8 channels.
__global__ void k_input(const float* x, int64_t n, bf16_t* t) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint4 z = make_uint4(0, 0, 0, 0);
    *(uint4*)(t + i * 8) = z;
    t[i * 8] = f2bf(x[i]);
}

// Head: out[v] = sum_ci y[v][ci] w[ci] + b (fp32); C is a multiple of 8,
// read 8 channels (16 bytes) at a time.
__global__ void k_head(const bf16_t* y, int C, const float* w, const float* b, int64_t n, float* out) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    float s = b[0];
    for (int c = 0; c < C; c += 8) {
        uint4 raw = *(const uint4*)(y + v * C + c);
        const bf16_t* h = (const bf16_t*)&raw;
#pragma unroll
        for (int j = 0; j < 8; ++j) s += bf2f(h[j]) * w[c + j];
    }
    out[v] = s;
}

// MSE loss: dout = 2 (out - target) / n; per-block partial sums of the
// squared error.
__global__ void k_mse(const float* out, const float* target, int64_t n, float* dout, float* part) {
    __shared__ float sh[4];
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float e = 0.f;
    if (i < n) {
        float d = out[i] - target[i];
        dout[i] = 2.f * d / (float)n;
        e = d * d;
    }
    float t = pic::block_sum(e, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Head backward: dy[v][c] = dout[v] w[c]; partials of dw[c] = sum dout y and db.
__global__ void k_head_back(const bf16_t* y, int C, const float* w, const float* dout, int64_t n, float* dy,
                            float* part) {
    __shared__ float sh[4];
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float d = v < n ? dout[v] : 0.f;
    for (int c = 0; c < C; ++c) {
        float yc = v < n ? bf2f(y[v * C + c]) : 0.f;
        if (v < n) dy[v * C + c] = d * w[c];
        float t = pic::block_sum(d * yc, sh);
        if (threadIdx.x == 0) part[(int64_t)blockIdx.x * (C + 1) + c] = t;
    }
    float t = pic::block_sum(d, sh);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * (C + 1) + C] = t;
}

// The same for C = 16 channels: each thread reads its voxel's 16 channels in
// two 16-byte loads and writes dy in four, and the 17 sums of the block are
// formed together (wavefront butterflies, then the four wavefronts' values
// added in wave order by 17 threads), one barrier instead of seventeen pairs.
__global__ __launch_bounds__(256) void k_head_back16(const bf16_t* y, const float* w, const float* dout, int64_t n,
                                                     float* dy, float* part) {
    __shared__ float sh[4][17];
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = v < n;
    const float d = in ? dout[v] : 0.f;
    float yc[16];
    if (in) {
        const uint4 r0 = *(const uint4*)(y + v * 16), r1 = *(const uint4*)(y + v * 16 + 8);
        const uint32_t u[8] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            yc[2 * k] = __uint_as_float(u[k] << 16);
            yc[2 * k + 1] = __uint_as_float(u[k] & 0xFFFF0000u);
        }
        float4* o = (float4*)(dy + v * 16);
#pragma unroll
        for (int q = 0; q < 4; ++q) o[q] = make_float4(d * w[4 * q], d * w[4 * q + 1], d * w[4 * q + 2], d * w[4 * q + 3]);
    } else {
#pragma unroll
        for (int c = 0; c < 16; ++c) yc[c] = 0.f;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 17; ++c) {
        const float t = pic::wave_sum(c < 16 ? d * yc[c] : d);
        if (lane == 0) sh[wv][c] = t;
    }
    __syncthreads();
    if (threadIdx.x < 17) {
        float t = 0.f;
        for (int q = 0; q < 4; ++q) t += sh[q][threadIdx.x];
        part[(int64_t)blockIdx.x * 17 + threadIdx.x] = t;
    }
}

// out[c] = sum over rows of part[r][c]: one block per column, each thread
// adding a strided subset in row order, then a block reduction (fixed order).
__global__ void k_sum_cols(const float* part, int nrows, int ncols, float* out) {
    __shared__ float sh[4];
    const int c = blockIdx.x;
    float s = 0.f;
    for (int r = threadIdx.x; r < nrows; r += blockDim.x) s += part[(int64_t)r * ncols + c];
    float t = pic::block_sum(s, sh);
    if (threadIdx.x == 0) out[c] = t;
}

// Adam (fp32 master weights).
__global__ void k_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.f - b1) * gi;
    float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// bf16 weight copies from the fp32 master W[tap][ci][co].
// Forward B operand: Wf[co][k], k = tap * cin + ci (sliced: one [co][ci]
// block per tap, for the up convolution whose rows each use one tap).
// Input-gradient B operand: Wb[ci][k], k = tap * cout + co (sliced: one
// [ci][co] block per tap, for the down convolution). Rows padded to Kf / Kb.
__global__ void k_pack_w(const float* w, int taps, int cin, int cout, int Kf, int sf, int Kb, int sb, bf16_t* wf,
                         bf16_t* wb) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t nf = (int64_t)(sf ? taps : 1) * cout * Kf, nb = (int64_t)(sb ? taps : 1) * cin * Kb;
    if (i < nf) {
        float val = 0.f;
        if (sf) {
            int t = (int)(i / ((int64_t)cout * Kf));
            int64_t r = i % ((int64_t)cout * Kf);
            int co = (int)(r / Kf), ci = (int)(r % Kf);
            if (ci < cin) val = w[((int64_t)t * cin + ci) * cout + co];
        } else {
            int co = (int)(i / Kf), k = (int)(i % Kf);
            if (k < taps * cin) val = w[((int64_t)(k / cin) * cin + (k % cin)) * cout + co];
        }
        wf[i] = f2bf(val);
    }
    if (i < nb) {
        float val = 0.f;
        if (sb) {
            int t = (int)(i / ((int64_t)cin * Kb));
            int64_t r = i % ((int64_t)cin * Kb);
            int ci = (int)(r / Kb), co = (int)(r % Kb);
            if (co < cout) val = w[((int64_t)t * cin + ci) * cout + co];
        } else {
            int ci = (int)(i / Kb), k = (int)(i % Kb);
            if (k < taps * cout) val = w[((int64_t)(k / cout) * cin + ci) * cout + (k % cout)];
        }
        wb[i] = f2bf(val);
    }
}

// g_a[v][0..ca) += t[v][0..ca), g_b[v][0..cb) += t[v][ca..ca+cb)
__global__ void k_split_add(const float* t, int64_t nvox, int ca, int cb, float* ga, float* gb) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int c = ca + cb;
    if (i >= nvox * c) return;
    int64_t v = i / c;
    int ch = (int)(i % c);
    if (ch < ca) ga[v * ca + ch] += t[i];
    else gb[v * cb + (ch - ca)] += t[i];
}

__global__ void k_copy_f32(const float* a, float* b, int64_t n, float scale) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i] * scale;
}

}  // namespace unet_impl

// ---------------------------------------------------------------------------
// Host side

using namespace unet_impl;

struct UnetLayer {
    int mode, ca, cb, cout, taps, relu;
    int64_t w_off, b_off;     // into the parameter vector
    int Kf, Kb;
    bf16_t *wf, *wb;          // bf16 copies
    int in_a, in_b, out;      // activation tensor indices (-1 none)
    Geo g;                    // GEMM row grid and input grid
};

struct unet {
    pic_unet_config cfg;
    hipStream_t stream;
    int B, D, H, W;
    float* params;
    float* grads;
    float *adam_m, *adam_v;
    int64_t nparams;
    int64_t adam_t;
    std::vector<UnetLayer> L;
    // activation tensors: bf16 values, fp32 gradients
    std::vector<bf16_t*> act;
    std::vector<float*> gact;
    std::vector<int> act_c;
    std::vector<int64_t> act_n;   // voxels
    int in_t, head_in;
    int64_t head_w, head_b;
    float *out, *dout;
    bf16_t* G;                    // masked gradient (bf16) scratch
    float* gm32;                  // masked gradient (fp32) scratch
    float* tmp32;                 // input gradient of a concatenating layer before the split
    float* part;                  // partial sums
    int64_t part_n;
    float* loss_part;
    char* ws;
    size_t ws_bytes, ws_used;
    std::string err;
};

static char* ws_take(unet* u, size_t bytes) {
    size_t off = (u->ws_used + 255) & ~size_t(255);
    if (off + bytes > u->ws_bytes) return nullptr;
    u->ws_used = off + bytes;
    return u->ws + off;
}

struct Plan {
    std::vector<UnetLayer> L;
    std::vector<int> act_c;
    std::vector<int64_t> act_n;
    int64_t nparams = 0;
    int head_in = -1, in_t = 0;
    int64_t head_w = 0, head_b = 0;
};

static Plan make_plan(const pic_unet_config* c, int B, int D, int H, int W) {
    Plan p;
    int ch[4] = {c->base_channels, 2 * c->base_channels, 4 * c->base_channels, 8 * c->base_channels};
    auto tensor = [&](int C, int64_t vox) {
        p.act_c.push_back(C);
        p.act_n.push_back(vox);
        return (int)p.act_c.size() - 1;
    };
    int64_t vox[4];
    int dims[4][3];
    for (int l = 0; l < 4; ++l) {
        dims[l][0] = D >> l;
        dims[l][1] = H >> l;
        dims[l][2] = W >> l;
        vox[l] = (int64_t)B * dims[l][0] * dims[l][1] * dims[l][2];
    }
    auto geo = [&](int lo, int li) {
        Geo g;
        g.B = B;
        g.D = dims[lo][0];
        g.H = dims[lo][1];
        g.W = dims[lo][2];
        g.iD = dims[li][0];
        g.iH = dims[li][1];
        g.iW = dims[li][2];
        return g;
    };
    auto add = [&](int mode, int a, int b, int cout, int relu, int lo, int li) {
        UnetLayer y;
        y.mode = mode;
        y.ca = p.act_c[a];
        y.cb = b >= 0 ? p.act_c[b] : 0;
        y.cout = cout;
        y.taps = mode == kModeSame3 ? 27 : 8;
        y.relu = relu;
        y.in_a = a;
        y.in_b = b;
        y.w_off = p.nparams;
        p.nparams += (int64_t)y.taps * (y.ca + y.cb) * cout;
        y.b_off = p.nparams;
        p.nparams += cout;
        int cin = y.ca + y.cb;
        y.Kf = (mode == kModeUp2 ? cin : y.taps * cin);      // per slice for the up convolution
        y.Kf = (y.Kf + 31) / 32 * 32;
        y.Kb = (mode == kModeDown2 ? cout : y.taps * cout);  // per slice for the down convolution
        y.Kb = (y.Kb + 31) / 32 * 32;
        int lo_t = mode == kModeUp2 ? li : lo;  // GEMM rows of the up conv are coarse voxels
        y.g = geo(lo_t, li);
        y.out = tensor(cout, vox[lo]);
        p.L.push_back(y);
        return y.out;
    };
    p.in_t = tensor(8, vox[0]);
    int x = add(kModeSame3, p.in_t, -1, ch[0], 1, 0, 0);
    int s0 = add(kModeSame3, x, -1, ch[0], 1, 0, 0);
    x = add(kModeDown2, s0, -1, ch[1], 1, 1, 0);
    x = add(kModeSame3, x, -1, ch[1], 1, 1, 1);
    int s1 = add(kModeSame3, x, -1, ch[1], 1, 1, 1);
    x = add(kModeDown2, s1, -1, ch[2], 1, 2, 1);
    x = add(kModeSame3, x, -1, ch[2], 1, 2, 2);
    int s2 = add(kModeSame3, x, -1, ch[2], 1, 2, 2);
    x = add(kModeDown2, s2, -1, ch[3], 1, 3, 2);
    x = add(kModeSame3, x, -1, ch[3], 1, 3, 3);
    x = add(kModeSame3, x, -1, ch[3], 1, 3, 3);
    x = add(kModeUp2, x, -1, ch[2], 0, 2, 3);
    x = add(kModeSame3, x, s2, ch[2], 1, 2, 2);
    x = add(kModeSame3, x, -1, ch[2], 1, 2, 2);
    x = add(kModeUp2, x, -1, ch[1], 0, 1, 2);
    x = add(kModeSame3, x, s1, ch[1], 1, 1, 1);
    x = add(kModeSame3, x, -1, ch[1], 1, 1, 1);
    x = add(kModeUp2, x, -1, ch[0], 0, 0, 1);
    x = add(kModeSame3, x, s0, ch[0], 1, 0, 0);
    x = add(kModeSame3, x, -1, ch[0], 1, 0, 0);
    p.head_in = x;
    p.head_w = p.nparams;
    p.nparams += ch[0];
    p.head_b = p.nparams;
    p.nparams += 1;
    return p;
}

// Layers whose weight gradient takes the one-pass kernel k_wgrad3 (staged
// channels ch a block, chunks of them along y), and its block count (one
// partial sum set each)
static bool wgrad3_pick(int mode, int taps, int cin, int N, int* ch) {
    if (mode != kModeSame3 || taps != 27) return false;
    if (cin == 8 && (N == 16 || N == 32)) *ch = 8;
    else if ((N == 16 || N == 32) && cin % 32 == 0) *ch = 32;
    else if ((N == 16 || N == 32 || N == 64) && cin % 16 == 0) *ch = 16;
    else return false;
    return true;
}
static bool wgrad3_ok(int mode, int taps, int cin, int N) {
    int ch;
    return wgrad3_pick(mode, taps, cin, N, &ch);
}
static int64_t wgrad3_blocks(const Geo& g) {  // at least two tiles a block
    return std::max<int64_t>(1, std::min<int64_t>(1024, conv3_tiles(g) / 2));
}

static int64_t wgrad_splits(int64_t M) {
    int64_t s = (M + 511) / 512;  // (small levels: enough blocks to fill the GPU)
    return s < 1 ? 1 : (s > 256 ? 256 : s);
}

static size_t plan_bytes(const Plan& p, int64_t vox0) {
    size_t b = 0;
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    for (size_t i = 0; i < p.act_c.size(); ++i) {
        b += al((size_t)p.act_n[i] * p.act_c[i] * 2);
        b += al((size_t)p.act_n[i] * p.act_c[i] * 4);
    }
    int64_t maxe = 0, maxpart = 0;
    for (const UnetLayer& y : p.L) {
        b += al((size_t)(y.mode == kModeUp2 ? 8 : 1) * y.cout * y.Kf * 2) +
             al((size_t)(y.mode == kModeDown2 ? 8 : 1) * (y.ca + y.cb) * y.Kb * 2);
        int64_t rows = (int64_t)y.g.B * y.g.D * y.g.H * y.g.W;
        maxe = std::max<int64_t>(maxe, (y.mode == kModeUp2 ? 8 * rows : rows) * std::max(y.cout, y.ca + y.cb));
        int64_t taps = y.mode == kModeUp2 ? 8 : y.taps;
        maxpart = std::max<int64_t>(maxpart, wgrad_splits(rows) * taps * (y.ca + y.cb) * y.cout);
        if (wgrad3_ok(y.mode, (int)taps, y.ca + y.cb, y.cout))
            maxpart = std::max<int64_t>(maxpart, wgrad3_blocks(y.g) * 27 * (y.ca + y.cb) * y.cout);
    }
    maxpart = std::max<int64_t>(maxpart, std::max<int64_t>(((vox0 + 255) / 256) * 64, 1024 * 128));
    b += al(maxe * 2) + 2 * al(maxe * 4) + al(maxpart * 4) + 2 * al(p.nparams * 4) + 2 * al(vox0 * 4) +
         al(((vox0 + 255) / 256 + 1) * 4) + 4096;
    return b;
}

static unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

static void launch_conv(unet* u, const UnetLayer& y, const bf16_t* a, const bf16_t* b, const bf16_t* w, int ca, int cb,
                        int N, int K, int Kpad, int mode, int relu, int flip, int par, Geo g, const float* bias,
                        bf16_t* out, float* out32, int accumulate) {
    ConvArgs p;
    p.a = a;
    p.b = b;
    p.w = w;
    p.bias = bias;
    p.out = out;
    p.out32 = out32;
    p.accumulate = accumulate;
    p.ca = ca;
    p.cb = cb;
    p.N = N;
    p.K = K;
    p.Kpad = Kpad;
    p.mode = mode;
    p.relu = relu;
    p.flip = flip;
    p.par = par;
    p.g = g;
    int64_t M = (int64_t)g.B * g.D * g.H * g.W;
    const int cin = ca + cb;
    // every input-channel count here is 8 or a multiple of 32 (chunks of 32)
    if (mode == kModeSame3 && (cin == 8 || cin == 16 || cin % kChunk == 0) &&
        (N == 16 || N == 32 || N == 64 || N == 128)) {
        const unsigned T = (unsigned)conv3_tiles(g);
        const int ch = cin < kChunk ? cin : kChunk;
        if ((cin == 8 || cin == 16) && (N == 16 || N == 32) && Kpad >= 27 * cin) {
            // persistent blocks, at least two tiles each (about the blocks
            // resident at once on the large levels)
            const dim3 grid(std::max(1u, std::min(T / 2, 1024u)), (unsigned)(N / 16));
            if (cin == 8) hipLaunchKernelGGL((k_conv3_ps<1, 8>), grid, dim3(256), 0, u->stream, p);
            else hipLaunchKernelGGL((k_conv3_ps<1, 16>), grid, dim3(256), 0, u->stream, p);
            return;
        }
        // output-channel groups: split while the grid has fewer than 512 blocks
        int nb = N / 16, split = 1;
        while (nb > 1 && T * split < 512u) {
            nb /= 2;
            split *= 2;
        }
#define CONV3_CH(NB)                                                                                       \
    (ch == 8 ? k_conv3_ch<NB, 8> : ch == 16 ? k_conv3_ch<NB, 16> : k_conv3_ch<NB, 32>)
        const dim3 grid(T, (unsigned)split);
        switch (nb) {
            case 1: hipLaunchKernelGGL(CONV3_CH(1), grid, dim3(256), 0, u->stream, p); break;
            case 2: hipLaunchKernelGGL(CONV3_CH(2), grid, dim3(256), 0, u->stream, p); break;
            case 4: hipLaunchKernelGGL(CONV3_CH(4), grid, dim3(256), 0, u->stream, p); break;
            default: hipLaunchKernelGGL(CONV3_CH(8), grid, dim3(256), 0, u->stream, p); break;
        }
#undef CONV3_CH
        return;
    }
    unsigned G = nblk(M, 64);
    switch (N / 16) {
        case 1: hipLaunchKernelGGL(k_conv<1>, dim3(G), dim3(256), 0, u->stream, p); break;
        case 2: hipLaunchKernelGGL(k_conv<2>, dim3(G), dim3(256), 0, u->stream, p); break;
        case 4: hipLaunchKernelGGL(k_conv<4>, dim3(G), dim3(256), 0, u->stream, p); break;
        case 8: hipLaunchKernelGGL(k_conv<8>, dim3(G), dim3(256), 0, u->stream, p); break;
        default: u->err = "unsupported channel count"; break;
    }
    (void)y;
}

static void pack_weights(unet* u) {
    for (UnetLayer& y : u->L) {
        int cin = y.ca + y.cb;
        int sf = y.mode == kModeUp2, sb = y.mode == kModeDown2;
        int64_t n = std::max<int64_t>((int64_t)(sf ? 8 : 1) * y.cout * y.Kf, (int64_t)(sb ? 8 : 1) * cin * y.Kb);
        hipLaunchKernelGGL(k_pack_w, dim3(nblk(n)), dim3(256), 0, u->stream, u->params + y.w_off, y.taps, cin, y.cout,
                           y.Kf, sf, y.Kb, sb, y.wf, y.wb);
    }
}

extern "C" {

pic_status unet_param_count(const pic_unet_config* c, int64_t* n) {
    if (!c || !n || c->base_channels < 16 || c->base_channels % 16 != 0 || c->base_channels > 16) return PIC_E_INVALID_ARG;
    Plan p = make_plan(c, 1, 8, 8, 8);
    *n = p.nparams;
    return PIC_OK;
}

pic_status unet_workspace_size(const pic_unet_config* c, int batch, int d, int h, int w, size_t* bytes) {
    if (!c || !bytes || batch < 1 || d < 8 || h < 8 || w < 8 || d % 8 || h % 8 || w % 8) return PIC_E_INVALID_ARG;
    if ((int64_t)batch * d * h * w >= ((int64_t)1 << 31)) return PIC_E_INVALID_ARG;  // 32-bit voxel indices
    if (c->base_channels != 16) return PIC_E_INVALID_ARG;
    Plan p = make_plan(c, batch, d, h, w);
    *bytes = plan_bytes(p, (int64_t)batch * d * h * w);
    return PIC_OK;
}

pic_status unet_create(const pic_unet_config* c, float* params, float* grads, void* workspace, size_t ws_bytes,
                       int batch, int d, int h, int w, void* stream, unet** out) {
    if (!out) return PIC_E_INVALID_ARG;
    *out = nullptr;
    size_t need = 0;
    if (unet_workspace_size(c, batch, d, h, w, &need) != PIC_OK || !params || !grads || !workspace || ws_bytes < need ||
        ((uintptr_t)workspace) % 256)
        return PIC_E_INVALID_ARG;
    unet* u = new unet();
    u->cfg = *c;
    u->stream = (hipStream_t)stream;
    u->B = batch;
    u->D = d;
    u->H = h;
    u->W = w;
    u->params = params;
    u->grads = grads;
    u->ws = (char*)workspace;
    u->ws_bytes = ws_bytes;
    u->ws_used = 0;
    Plan p = make_plan(c, batch, d, h, w);
    u->L = p.L;
    u->act_c = p.act_c;
    u->act_n = p.act_n;
    u->nparams = p.nparams;
    u->head_in = p.head_in;
    u->in_t = p.in_t;
    u->head_w = p.head_w;
    u->head_b = p.head_b;
    for (size_t i = 0; i < p.act_c.size(); ++i) {
        u->act.push_back((bf16_t*)ws_take(u, (size_t)p.act_n[i] * p.act_c[i] * 2));
        u->gact.push_back((float*)ws_take(u, (size_t)p.act_n[i] * p.act_c[i] * 4));
    }
    int64_t maxe = 0, maxpart = 0;
    for (UnetLayer& y : u->L) {
        y.wf = (bf16_t*)ws_take(u, (size_t)(y.mode == kModeUp2 ? 8 : 1) * y.cout * y.Kf * 2);
        y.wb = (bf16_t*)ws_take(u, (size_t)(y.mode == kModeDown2 ? 8 : 1) * (y.ca + y.cb) * y.Kb * 2);
        int64_t rows = (int64_t)y.g.B * y.g.D * y.g.H * y.g.W;
        maxe = std::max<int64_t>(maxe, (y.mode == kModeUp2 ? 8 * rows : rows) * std::max(y.cout, y.ca + y.cb));
        int64_t taps = y.mode == kModeUp2 ? 8 : y.taps;
        maxpart = std::max<int64_t>(maxpart, wgrad_splits(rows) * taps * (y.ca + y.cb) * y.cout);
        if (wgrad3_ok(y.mode, (int)taps, y.ca + y.cb, y.cout))
            maxpart = std::max<int64_t>(maxpart, wgrad3_blocks(y.g) * 27 * (y.ca + y.cb) * y.cout);
    }
    int64_t vox0 = (int64_t)batch * d * h * w;
    maxpart = std::max<int64_t>(maxpart, std::max<int64_t>(((vox0 + 255) / 256) * 64, 1024 * 128));
    u->G = (bf16_t*)ws_take(u, maxe * 2);
    u->gm32 = (float*)ws_take(u, maxe * 4);
    u->tmp32 = (float*)ws_take(u, maxe * 4);
    u->part = (float*)ws_take(u, maxpart * 4);
    u->part_n = maxpart;
    u->adam_m = (float*)ws_take(u, u->nparams * 4);
    u->adam_v = (float*)ws_take(u, u->nparams * 4);
    u->out = (float*)ws_take(u, vox0 * 4);
    u->dout = (float*)ws_take(u, vox0 * 4);
    u->loss_part = (float*)ws_take(u, ((vox0 + 255) / 256 + 1) * 4);
    if (!u->loss_part) {
        delete u;
        return PIC_E_INVALID_ARG;
    }
    (void)pic::launch_zero(u->adam_m, u->nparams * 4, u->stream);
    (void)pic::launch_zero(u->adam_v, u->nparams * 4, u->stream);
    u->adam_t = 0;
    pack_weights(u);
    if (hipGetLastError() != hipSuccess) {
        delete u;
        return PIC_E_HIP;
    }
    *out = u;
    return PIC_OK;
}

// Forward: x (fp32, [batch][d][h][w]) -> y (fp32, same shape). The weights
// are read from the parameter vector as last packed (unet_create,
// unet_adam_step, unet_sync_params).
pic_status unet_forward(unet* u, const float* x, float* y) {
    if (!u || !x) return PIC_E_INVALID_ARG;
    int64_t n0 = u->act_n[u->in_t];
    hipLaunchKernelGGL(k_input, dim3(nblk(n0)), dim3(256), 0, u->stream, x, n0, u->act[u->in_t]);
    for (const UnetLayer& l : u->L) {
        const bf16_t* a = u->act[l.in_a];
        const bf16_t* b = l.in_b >= 0 ? u->act[l.in_b] : nullptr;
        int cin = l.ca + l.cb;
        const float* bias = u->params + l.b_off;
        if (l.mode == kModeUp2 && l.Kf == cin && ((l.cout == 16 && cin == 32) || (l.cout == 32 && cin == 64) ||
                                                  (l.cout == 64 && cin == 128))) {
            // the eight parities in one launch (the argument set of launch_conv)
            ConvArgs p{};
            p.a = a;
            p.b = b;
            p.w = l.wf;
            p.bias = bias;
            p.out = u->act[l.out];
            p.ca = l.ca;
            p.cb = l.cb;
            p.N = l.cout;
            p.K = cin;
            p.Kpad = l.Kf;
            p.mode = kModeUp2;
            p.relu = l.relu;
            p.g = l.g;
            const int64_t M = (int64_t)l.g.B * l.g.D * l.g.H * l.g.W;
            const unsigned G = nblk(M, 64);
            if (l.cout == 16) hipLaunchKernelGGL((k_up2_all<1, 1>), dim3(G), dim3(256), 0, u->stream, p);
            else if (l.cout == 32) hipLaunchKernelGGL((k_up2_all<2, 2>), dim3(G), dim3(256), 0, u->stream, p);
            else hipLaunchKernelGGL((k_up2_all<4, 4>), dim3(G), dim3(256), 0, u->stream, p);
        } else if (l.mode == kModeUp2) {
            for (int par = 0; par < 8; ++par)
                launch_conv(u, l, a, b, l.wf + (int64_t)par * l.cout * l.Kf, l.ca, l.cb, l.cout, cin, l.Kf, kModeUp2,
                            l.relu, 0, par, l.g, bias, u->act[l.out], nullptr, 0);
        } else {
            launch_conv(u, l, a, b, l.wf, l.ca, l.cb, l.cout, l.taps * cin, l.Kf, l.mode, l.relu, 0, 0, l.g, bias,
                        u->act[l.out], nullptr, 0);
        }
    }
    hipLaunchKernelGGL(k_head, dim3(nblk(n0)), dim3(256), 0, u->stream, u->act[u->head_in], u->act_c[u->head_in],
                       u->params + u->head_w, u->params + u->head_b, n0, u->out);
    if (y) hipLaunchKernelGGL(k_copy_f32, dim3(nblk(n0)), dim3(256), 0, u->stream, u->out, y, n0, 1.0f);
    return hipGetLastError() == hipSuccess && u->err.empty() ? PIC_OK : PIC_E_HIP;
}

}  // extern "C"

static void launch_wgrad(unet* u, const UnetLayer& l, const bf16_t* a, const bf16_t* b, int taps, int par, Geo g,
                         float* dst) {
    WgradArgs w;
    w.a = a;
    w.b = b;
    w.gr = u->G;
    w.part = u->part;
    w.ca = l.ca;
    w.cb = l.cb;
    w.N = l.cout;
    w.taps = taps;
    w.mode = l.mode;
    w.par = par;
    w.g = g;
    int64_t rows = (int64_t)g.B * g.D * g.H * g.W;
    const int cin = l.ca + l.cb;
    int ch = 0;
    if (wgrad3_pick(l.mode, taps, cin, l.cout, &ch)) {
        const int64_t nb = wgrad3_blocks(g);
        const dim3 G((unsigned)nb, (unsigned)(cin / ch));
        const int nt = l.cout / 16;
        if (ch == 8) {
            if (nt == 1) hipLaunchKernelGGL((k_wgrad3<8, 1>), G, dim3(256), 0, u->stream, w);
            else hipLaunchKernelGGL((k_wgrad3<8, 2>), G, dim3(256), 0, u->stream, w);
        } else if (ch == 16) {
            if (nt == 1) hipLaunchKernelGGL((k_wgrad3<16, 1>), G, dim3(256), 0, u->stream, w);
            else if (nt == 2) hipLaunchKernelGGL((k_wgrad3<16, 2>), G, dim3(256), 0, u->stream, w);
            else hipLaunchKernelGGL((k_wgrad3<16, 4>), G, dim3(256), 0, u->stream, w);
        } else {
            if (nt == 1) hipLaunchKernelGGL((k_wgrad3<32, 1>), G, dim3(256), 0, u->stream, w);
            else hipLaunchKernelGGL((k_wgrad3<32, 2>), G, dim3(256), 0, u->stream, w);
        }
        const int64_t n = (int64_t)27 * cin * l.cout;
        hipLaunchKernelGGL(k_sum_splits, dim3(nblk(n)), dim3(256), 0, u->stream, (const float*)u->part, (int)nb, n,
                           dst);
        return;
    }
    int64_t ns = wgrad_splits(rows);
    w.rows_per_split = (rows + ns - 1) / ns;
    const int cin16 = (l.ca + l.cb + 15) / 16 * 16;
    if (cin16 <= 64 && l.cout <= 64)
        hipLaunchKernelGGL(k_wgrad2<128>, dim3((unsigned)(ns * taps)), dim3(256), 0, u->stream, w);
    else
        hipLaunchKernelGGL(k_wgrad2<32>, dim3((unsigned)(ns * taps)), dim3(256), 0, u->stream, w);
    int64_t n = (int64_t)taps * (l.ca + l.cb) * l.cout;
    hipLaunchKernelGGL(k_sum_splits, dim3(nblk(n)), dim3(256), 0, u->stream, (const float*)u->part, (int)ns, n, dst);
}

extern "C" {

// Backward of the last forward against target (fp32, same shape as the
// output): MSE loss, gradients of every parameter into the gradient vector.
// loss (host, optional) receives the mean squared error (synchronizes).
pic_status unet_backward(unet* u, const float* target, double* loss) {
    if (!u || !target) return PIC_E_INVALID_ARG;
    int64_t n0 = u->act_n[u->in_t];
    unsigned nb0 = nblk(n0);
    hipLaunchKernelGGL(k_mse, dim3(nb0), dim3(256), 0, u->stream, (const float*)u->out, target, n0, u->dout,
                       u->loss_part);
    for (size_t i = 0; i < u->act.size(); ++i)
        (void)pic::launch_zero(u->gact[i], (size_t)u->act_n[i] * u->act_c[i] * 4, u->stream);
    int Ch = u->act_c[u->head_in];
    if (Ch == 16)
        hipLaunchKernelGGL(k_head_back16, dim3(nb0), dim3(256), 0, u->stream, (const bf16_t*)u->act[u->head_in],
                           u->params + u->head_w, (const float*)u->dout, n0, u->gact[u->head_in], u->part);
    else
        hipLaunchKernelGGL(k_head_back, dim3(nb0), dim3(256), 0, u->stream, (const bf16_t*)u->act[u->head_in], Ch,
                       (const float*)(u->params + u->head_w), (const float*)u->dout, n0, u->gact[u->head_in], u->part);
    hipLaunchKernelGGL(k_sum_cols, dim3(Ch + 1), dim3(256), 0, u->stream, (const float*)u->part, (int)nb0, Ch + 1,
                       u->grads + u->head_w);  // head_b follows head_w
    for (int li = (int)u->L.size() - 1; li >= 0; --li) {
        const UnetLayer& l = u->L[li];
        int64_t nout = u->act_n[l.out] * l.cout;
        hipLaunchKernelGGL(k_mask, dim3(nblk(nout)), dim3(256), 0, u->stream, (const float*)u->gact[l.out],
                           (const bf16_t*)u->act[l.out], l.relu, nout, u->G, u->gm32);
        // bias
        int nbb = 1024;
        hipLaunchKernelGGL(k_bias_partial, dim3(nbb), dim3(256), 0, u->stream, (const float*)u->gm32, u->act_n[l.out],
                           l.cout, u->part);
        hipLaunchKernelGGL(k_sum_cols, dim3(l.cout), dim3(256), 0, u->stream, (const float*)u->part, nbb, l.cout,
                           u->grads + l.b_off);
        const bf16_t* a = u->act[l.in_a];
        const bf16_t* b = l.in_b >= 0 ? u->act[l.in_b] : nullptr;
        int cin = l.ca + l.cb;
        // weights
        if (l.mode == kModeUp2) {
            for (int par = 0; par < 8; ++par)
                launch_wgrad(u, l, a, b, 1, par, l.g, u->grads + l.w_off + (int64_t)par * cin * l.cout);
        } else {
            launch_wgrad(u, l, a, b, l.taps, 0, l.g, u->grads + l.w_off);
        }
        // input gradient
        if (l.in_a == u->in_t) continue;
        if (l.mode == kModeSame3) {
            Geo g = l.g;  // same grid in and out
            float* dst = l.in_b >= 0 ? u->tmp32 : u->gact[l.in_a];
            launch_conv(u, l, u->G, nullptr, l.wb, l.cout, 0, cin, 27 * l.cout, l.Kb, kModeSame3, 0, 1, 0, g, nullptr,
                        nullptr, dst, l.in_b >= 0 ? 0 : 1);
            if (l.in_b >= 0) {
                int64_t nv = u->act_n[l.in_a];
                hipLaunchKernelGGL(k_split_add, dim3(nblk(nv * cin)), dim3(256), 0, u->stream, (const float*)u->tmp32, nv,
                                   l.ca, l.cb, u->gact[l.in_a], u->gact[l.in_b]);
            }
        } else if (l.mode == kModeDown2) {
            // rows: coarse voxels of the output; each parity writes its fine voxels
            Geo g = l.g;
            g.iD = g.D;
            g.iH = g.H;
            g.iW = g.W;
            for (int par = 0; par < 8; ++par)
                launch_conv(u, l, u->G, nullptr, l.wb + (int64_t)par * cin * l.Kb, l.cout, 0, cin, l.cout, l.Kb,
                            kModeUp2, 0, 0, par, g, nullptr, nullptr, u->gact[l.in_a], 1);
        } else {
            // up convolution: coarse input gradient from the 8 fine children
            Geo g = l.g;
            g.iD = 2 * g.D;
            g.iH = 2 * g.H;
            g.iW = 2 * g.W;
            launch_conv(u, l, u->G, nullptr, l.wb, l.cout, 0, cin, 8 * l.cout, l.Kb, kModeDown2, 0, 0, 0, g, nullptr,
                        nullptr, u->gact[l.in_a], 1);
        }
    }
    if (loss) {
        std::vector<float> h(nb0);
        if (hipMemcpyAsync(h.data(), u->loss_part, nb0 * 4, hipMemcpyDeviceToHost, u->stream) != hipSuccess ||
            hipStreamSynchronize(u->stream) != hipSuccess)
            return PIC_E_HIP;
        double s = 0.0;
        for (unsigned i = 0; i < nb0; ++i) s += h[i];
        *loss = s / (double)n0;
    }
    return hipGetLastError() == hipSuccess && u->err.empty() ? PIC_OK : PIC_E_HIP;
}

// One Adam step on the fp32 master weights with the current gradients, then
// the bf16 copies are refreshed.
pic_status unet_adam_step(unet* u, float lr, float beta1, float beta2, float eps) {
    if (!u || !(lr > 0)) return PIC_E_INVALID_ARG;
    u->adam_t += 1;
    float c1 = 1.f - powf(beta1, (float)u->adam_t), c2 = 1.f - powf(beta2, (float)u->adam_t);
    hipLaunchKernelGGL(k_adam, dim3(nblk(u->nparams)), dim3(256), 0, u->stream, u->params, (const float*)u->grads,
                       u->adam_m, u->adam_v, u->nparams, lr, beta1, beta2, eps, c1, c2);
    pack_weights(u);
    return hipGetLastError() == hipSuccess ? PIC_OK : PIC_E_HIP;
}

// Refresh the bf16 weight copies after the caller changed the parameters.
pic_status unet_sync_params(unet* u) {
    if (!u) return PIC_E_INVALID_ARG;
    pack_weights(u);
    return hipGetLastError() == hipSuccess ? PIC_OK : PIC_E_HIP;
}

void unet_destroy(unet* u) {
    if (!u) return;
    (void)hipStreamSynchronize(u->stream);
    delete u;
}

}  // extern "C"


// ---------------------------------------------------------------------------
// Learned warm start and training pairs of a context.

namespace pic {

constexpr double kTwoM40 = 9.094947017729282379e-13;  // 2^-40

// max |rho| per block (integer, exact)
__global__ void k_absmax_part(const int64_t* __restrict__ rho, int64_t n, unsigned long long* part) {
    unsigned long long m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t v = rho[i];
        unsigned long long a = (unsigned long long)(v < 0 ? -v : v);
        m = a > m ? a : m;
    }
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long t = __shfl_xor(m, o);
        m = t > m ? t : m;
    }
    __shared__ unsigned long long sh[kBlock / 64];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x / 64); ++w) m = sh[w] > m ? sh[w] : m;
        part[blockIdx.x] = m;
    }
}

__global__ void k_absmax_final(const unsigned long long* part, int nparts, DevState* st) {
    unsigned long long m = 0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) m = part[i] > m ? part[i] : m;
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long t = __shfl_xor(m, o);
        m = t > m ? t : m;
    }
    if (threadIdx.x == 0) st->learn_scale = (double)m * kTwoM40;
}

// x = q / s (zero without charge)
__global__ void k_learn_input(const int64_t* __restrict__ rho, int64_t n, const DevState* st, float* __restrict__ x) {
    double s = st->learn_scale;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = s > 0.0 ? (float)((double)rho[i] * kTwoM40 / s) : 0.f;
}

// yo = binomial [1 2 1]/4 filter of yi along x, y and z (edges replicated):
// removes the node-scale (checkerboard) part of the network's output, which
// the operator would otherwise turn into a large residual.
__global__ void k_learn_smooth(const float* __restrict__ yi, float* __restrict__ yo, int nx, int ny, int nz) {
    int64_t n = (int64_t)nx * ny * nz;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
        float acc = 0.f;
        for (int dz = -1; dz <= 1; ++dz) {
            int zz = min(max(z + dz, 0), nz - 1);
            float wz = dz == 0 ? 0.5f : 0.25f;
            for (int dy = -1; dy <= 1; ++dy) {
                int yy = min(max(y + dy, 0), ny - 1);
                float wy = dy == 0 ? 0.5f : 0.25f;
                for (int dx = -1; dx <= 1; ++dx) {
                    int xx = min(max(x + dx, 0), nx - 1);
                    float wx = dx == 0 ? 0.5f : 0.25f;
                    acc += wz * wy * wx * yi[((int64_t)zz * ny + yy) * nx + xx];
                }
            }
        }
        yo[i] = acc;
    }
}

// phi = V0 phi1 + gamma y on free nodes (gamma from st), V0 phi1 elsewhere,
// without a network output and when gamma is zero (which it is when the
// network output was not finite: 0 * NaN must not reach the guess)
__global__ void k_learn_phi(const double* __restrict__ phi1, const float* __restrict__ y, const uint8_t* __restrict__ type,
                            int64_t n, double V0, const DevState* st, double* __restrict__ phi) {
    const double gam = st->learn_gamma;
    const bool use_y = y && gam != 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double v = V0 * phi1[i];
        if (use_y && type[i] == 0) v += gam * (double)y[i];
        phi[i] = v;
    }
}

// Partials of y.q and y.(L y) over the free nodes, with y taken as zero on
// fixed nodes, L the finite-volume operator of Eq. poi and q = rho qscale its
// charge term. V0 phi1 satisfies the charge-free problem, so the residual of
// V0 phi1 + g y is q - g L y and g* = (y.q) / (y.L y) minimizes the energy
// norm of the error along y: the guess is never worse in that norm than V0
// phi1 alone.
__device__ inline double learn_half(int i, int n) { return (i == 0 || i == n - 1) ? 0.5 : 1.0; }

__global__ __launch_bounds__(kBlock) void k_learn_proj(Grid g, const float* __restrict__ y, const int64_t* __restrict__ rho,
                                                        const uint8_t* __restrict__ type, double qscale,
                                                        double* __restrict__ part) {
    const int64_t pl = (int64_t)g.nx * g.ny;
    double yq = 0.0, yly = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < g.nn; n += (int64_t)gridDim.x * blockDim.x) {
        if (type[n] != 0) continue;
        const int i = (int)(n % g.nx), j = (int)((n / g.nx) % g.ny), k = (int)(n / pl);
        const double fx = learn_half(j, g.ny) * learn_half(k, g.nz), fy = learn_half(i, g.nx) * learn_half(k, g.nz),
                     fz = learn_half(i, g.nx) * learn_half(j, g.ny);
        const double yn = y[n];
        const int64_t nb[6] = {n - 1, n + 1, n - g.nx, n + g.nx, n - pl, n + pl};
        const bool has[6] = {i > 0, i < g.nx - 1, j > 0, j < g.ny - 1, k > 0, k < g.nz - 1};
        const double f[6] = {fx, fx, fy, fy, fz, fz};
        double ly = 0.0;
        for (int d = 0; d < 6; ++d) {
            if (!has[d]) continue;
            const double ym = type[nb[d]] == 0 ? (double)y[nb[d]] : 0.0;
            ly += f[d] * (yn - ym);
        }
        yq += yn * ((double)rho[n] * qscale);
        yly += yn * ly;
    }
    __shared__ double sh[kBlock / 64];
    const double a = block_sum(yq, sh);
    __syncthreads();
    const double b = block_sum(yly, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

// gamma: the projection weight (project != 0), else the network's own
// scaling e s / (eps0 h); zero, with learn_bad set, when y.q or y.L y is not
// finite (a network output with NaN or infinity anywhere on a free node)
__global__ void k_learn_gamma(const double* __restrict__ part, int nparts, int project, double c0, DevState* st) {
    if (threadIdx.x != 0) return;
    double a = 0.0, b = 0.0;
    for (int i = 0; i < nparts; ++i) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    const bool bad = !isfinite(a) || !isfinite(b);
    st->learn_bad = bad ? 1 : 0;
    double g = project ? (b > 0.0 ? a / b : 0.0) : (st->learn_scale > 0.0 ? c0 * st->learn_scale : 0.0);
    st->learn_gamma = (bad || !isfinite(g)) ? 0.0 : g;
}

// y = (phi - V0 phi1) eps0 h / (e s) on free nodes, zero elsewhere
__global__ void k_learn_target(const double* __restrict__ phi, const double* __restrict__ phi1,
                               const uint8_t* __restrict__ type, int64_t n, double V0, double c1, const DevState* st,
                               float* __restrict__ y) {
    double s = st->learn_scale;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (s > 0.0 && type[i] == 0) ? (float)((phi[i] - V0 * phi1[i]) * c1 / s) : 0.f;
}

static hipError_t learn_scale_and_input(pic_ctx* c, float* x) {
    int64_t n = c->g.nn;
    unsigned G = 1024;
    unsigned long long* part = (unsigned long long*)c->partials;
    hipLaunchKernelGGL(k_absmax_part, dim3(G), dim3(kBlock), 0, c->stream, (const int64_t*)c->buf.rho, n, part);
    hipLaunchKernelGGL(k_absmax_final, dim3(1), dim3(64), 0, c->stream, (const unsigned long long*)part, (int)G, c->st);
    if (x) hipLaunchKernelGGL(k_learn_input, dim3(4096), dim3(kBlock), 0, c->stream, (const int64_t*)c->buf.rho, n,
                              (const pic::DevState*)c->st, x);
    return hipGetLastError();
}

int guess_phi(pic_ctx* c, bool with_net) {
    int64_t n = c->g.nn;
    const float* y = nullptr;
    if (with_net) {
        // network input and output in the (idle) CG work vectors
        float* x = (float*)c->cg_p0;
        float* yo = (float*)c->cg_q;
        if (learn_scale_and_input(c, x) != hipSuccess) return -2;
        if (unet_forward(c->learned, x, yo) != PIC_OK) return -2;
        float* a = yo;
        float* b = x;  // the input is no longer needed
        for (int k = 0; k < c->learn_smooth; ++k) {
            hipLaunchKernelGGL(k_learn_smooth, dim3(4096), dim3(kBlock), 0, c->stream, (const float*)a, b, c->cfg.nx,
                               c->cfg.ny, c->cfg.nz);
            std::swap(a, b);
        }
        y = a;
    }
    if (y) {
        const unsigned G = 256;
        double* part = c->partials;  // idle between solves
        const double qscale = ldexp(1.0, -40) * kQe / (kEps0 * c->cfg.h);
        hipLaunchKernelGGL(k_learn_proj, dim3(G), dim3(kBlock), 0, c->stream, c->g, y, (const int64_t*)c->buf.rho,
                           (const uint8_t*)c->buf.node_type, qscale, part);
        hipLaunchKernelGGL(k_learn_gamma, dim3(1), dim3(64), 0, c->stream, (const double*)part, (int)G,
                           c->learn_project, kQe / (kEps0 * c->cfg.h), c->st);
    }
    hipLaunchKernelGGL(k_learn_phi, dim3(4096), dim3(kBlock), 0, c->stream, (const double*)c->buf.phi1, y,
                       (const uint8_t*)c->buf.node_type, n, c->V0, (const pic::DevState*)c->st,
                       (double*)c->buf.phi);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace pic

extern "C" {

pic_status pic_set_learned_guess(pic_ctx* c, unet* u, int32_t smooth_passes, int32_t project, int32_t fallback) {
    if (!c || smooth_passes < 0 || smooth_passes > 64 || project < 0 || project > 1 || fallback < 0 || fallback > 1)
        return PIC_E_INVALID_ARG;
    if (u && (u->B != 1 || u->D != c->cfg.nz || u->H != c->cfg.ny || u->W != c->cfg.nx || u->stream != c->stream))
        return PIC_E_INVALID_ARG;
    c->learned = u;
    c->learn_smooth = smooth_passes;
    c->learn_project = project;
    c->learn_fallback = fallback;
    return PIC_OK;
}

pic_status pic_training_sample(pic_ctx* c, float* x, float* y, double* scale) {
    if (!c || !x || !y) return PIC_E_INVALID_ARG;
    if (c->failed) return PIC_E_STATE;
    if (pic::learn_scale_and_input(c, x) != hipSuccess) return PIC_E_HIP;
    double c1 = pic::kEps0 * c->cfg.h / pic::kQe;
    hipLaunchKernelGGL(pic::k_learn_target, dim3(4096), dim3(pic::kBlock), 0, c->stream, (const double*)c->buf.phi,
                       (const double*)c->buf.phi1, (const uint8_t*)c->buf.node_type, c->g.nn, c->V0, c1,
                       (const pic::DevState*)c->st, y);
    if (hipGetLastError() != hipSuccess) return PIC_E_HIP;
    if (scale) {
        double s = 0.0;
        if (hipMemcpyAsync(&s, &c->st->learn_scale, sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            return PIC_E_HIP;
        *scale = s;
    }
    return PIC_OK;
}

}  // extern "C"
