// particles.hip -- particle kernels of one PIC-MCC step: push with deposit and
// binning, cell bins, Monte Carlo collisions, field ionization, products,
// reordering by cell, field emission, explicit loads.
#include <algorithm>

#include "pic_internal.hpp"

namespace pic {

// ---------------------------------------------------------------------------
// Push (Sec. 2.2): gather of the node field at x^n by trilinear weights,
// leapfrog kick v^{n+1/2} = v^{n-1/2} + (q/m) E dt and drift
// x^{n+1} = x^n + v^{n+1/2} dt (neutrals drift); particles that end outside
// the vacuum region are removed. Fused with the rest of the per-particle pass
// over x^{n+1}:
//  - the cell key and the particle's slot among the particles of its cell;
//  - for neutrals, the field-ionization test of Eq. dfi at x^{n+1} (the draw
//    is keyed by particle id and step, so the test can run here; whether the
//    neutral is free to ionize is decided after the collisions);
//  - the largest speed per species (bound for the null-collision test).
// The charge deposit follows from the cell bins (k_deposit_tiles). Products
// of ionization carry +e and -e at the same point, so depositing before the
// collisions gives the same node charge as after them.

template <typename T>
struct PushArgs {
    Species<T> s;
    const typename V4<T>::type* field;
    Grid g;
    T kq;
    int64_t* rho;
    int64_t sign;
    uint32_t* key;   // cell key of each slot (kDead: no particle), binned by binning.hip
    DevState* st;
    uint32_t step;
    uint64_t seed;
    uint32_t* fi_list;
    uint32_t* part;  // per-block partials: [block][8] = max speed bits, lost[1..4], bsi
    double* dpart;   // per-block FP64 partials: [block][4] = sum |V|^2 of ions reaching the cathode plane and
                     // the tip, sum V . E0 (the Shockley-Ramo current before its factor)
    const typename V4<T>::type* field0;  // weighting field (with the circuit only, else null)
    uint32_t* fi_cnt;  // weighted runs: field-ionized units of each candidate neutral
    double fi_thr, ebsi, adk_c, adk_e, x32, dt_fs;
};

template <typename T>
__device__ inline void gather(const Grid& g, const typename V4<T>::type* __restrict__ E, T X, T Y, T Z, T& ex,
                              T& ey, T& ez) {
    int i = clampi((int)floor(X), 0, g.nx - 2);
    int j = clampi((int)floor(Y), 0, g.ny - 2);
    int k = clampi((int)floor(Z), 0, g.nz - 2);
    T fx = X - (T)i, fy = Y - (T)j, fz = Z - (T)k;
    T gx = (T)1 - fx, gy = (T)1 - fy, gz = (T)1 - fz;
    int64_t n0 = ((int64_t)k * g.ny + j) * g.nx + i;
    int64_t pl = (int64_t)g.nx * g.ny;
    auto e000 = E[n0], e100 = E[n0 + 1], e010 = E[n0 + g.nx], e110 = E[n0 + g.nx + 1];
    auto e001 = E[n0 + pl], e101 = E[n0 + pl + 1], e011 = E[n0 + pl + g.nx], e111 = E[n0 + pl + g.nx + 1];
    T w000 = gx * gy * gz, w100 = fx * gy * gz, w010 = gx * fy * gz, w110 = fx * fy * gz;
    T w001 = gx * gy * fz, w101 = fx * gy * fz, w011 = gx * fy * fz, w111 = fx * fy * fz;
    ex = w000 * e000.x + w100 * e100.x + w010 * e010.x + w110 * e110.x + w001 * e001.x + w101 * e101.x +
         w011 * e011.x + w111 * e111.x;
    ey = w000 * e000.y + w100 * e100.y + w010 * e010.y + w110 * e110.y + w001 * e001.y + w101 * e101.y +
         w011 * e011.y + w111 * e111.y;
    ez = w000 * e000.z + w100 * e100.z + w010 * e010.z + w110 * e110.z + w001 * e001.z + w101 * e101.z +
         w011 * e011.z + w111 * e111.z;
}

__device__ inline unsigned int speed_bits(double s) {
    float f = (float)s;
    if ((double)f < s) f = __uint_as_float(__float_as_uint(f) + 1u);  // next float up (s >= 0)
    return __float_as_uint(f);
}

template <typename T, int SP, bool MOVE>
__global__ __launch_bounds__(kBlock) void k_push(PushArgs<T> a) {
    const Grid& g = a.g;
    const int64_t n = (int64_t)a.st->n_slots[SP];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned int smax = 0;
    // removals per boundary and neutrals above the barrier-suppression field:
    // counted per thread, reduced per block (one atomic per block and kind)
    unsigned int lost[5] = {0, 0, 0, 0, 0};
    unsigned int bsi = 0;
    // ions reaching the cathode plane and the tip (bombardment, Sec. 2.3.3)
    // and the Shockley-Ramo sum of the pushed charges (Sec. 2.3.1)
    double bomb[2] = {0.0, 0.0};
    double sr = 0.0;
    // Lanes past the last slot load the last slot and store nothing, so the
    // loads need no branch.
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += stride) {
        const int64_t i = base + threadIdx.x;
        const bool valid = i < n;
        const int64_t il = valid ? i : n - 1;
        // The id and the state are loaded together and free slots go through
        // the same arithmetic (their results are not stored), so no branch
        // separates the loads: one memory latency for the state, one for the
        // gathered field.
        const uint32_t id = a.s.id[il];
        T X = a.s.x[il], Y = a.s.y[il], Z = a.s.z[il];
        T VX = a.s.vx[il], VY = a.s.vy[il], VZ = a.s.vz[il];
        const bool alive = valid && id != kDead;
        if (MOVE) {
            if (SP != PIC_NEUTRAL) {
                T ex, ey, ez;
                gather<T>(g, a.field, X, Y, Z, ex, ey, ez);
                VX += a.kq * ex;
                VY += a.kq * ey;
                VZ += a.kq * ez;
                if (a.field0) {
                    // the weighting field at x^n with v^{n+1/2}
                    T wx, wy, wz;
                    gather<T>(g, a.field0, X, Y, Z, wx, wy, wz);
                    if (alive)
                        sr += (a.s.w ? (double)a.s.w[il] : 1.0) *
                              ((double)VX * (double)wx + (double)VY * (double)wy + (double)VZ * (double)wz);
                }
            }
            X += VX;
            Y += VY;
            Z += VZ;
        }
        const double Xd = (double)X, Yd = (double)Y, Zd = (double)Z;
        const int code = alive ? boundary_code(g, Xd, Yd, Zd) : 0;
        const int ci = clampi((int)floor(Xd), 0, g.nx - 2);
        const int cj = clampi((int)floor(Yd), 0, g.ny - 2);
        const int ck = clampi((int)floor(Zd), 0, g.nz - 2);
        const bool keep = alive && code == 0;
        const uint32_t key = keep ? cell_key(g, ci, cj, ck) : kDead;
        if (valid) a.key[i] = key;
        if (!alive) continue;
        if (MOVE) {
            if (SP != PIC_NEUTRAL) {
                a.s.vx[i] = VX;
                a.s.vy[i] = VY;
                a.s.vz[i] = VZ;
            }
            a.s.x[i] = X;
            a.s.y[i] = Y;
            a.s.z[i] = Z;
        }
        if (code != 0) {
            a.s.id[i] = kDead;
            lost[code]++;
            if (SP == PIC_ION && MOVE && (code == 1 || code == 4)) {
                const double vx = (double)VX, vy = (double)VY, vz = (double)VZ;
                bomb[code == 1 ? 0 : 1] += (a.s.w ? (double)a.s.w[i] : 1.0) * (vx * vx + vy * vy + vz * vz);
            }
            continue;
        }
        double vx = (double)VX, vy = (double)VY, vz = (double)VZ;
        unsigned int sb = speed_bits(sqrt(vx * vx + vy * vy + vz * vz));
        smax = sb > smax ? sb : smax;
        if (SP == PIC_NEUTRAL) {
            // Field ionization of Eq. dfi: rate per fs at the local field in
            // GV/m; no attempt above the barrier-suppression field.
            T ex, ey, ez;
            gather<T>(g, a.field, X, Y, Z, ex, ey, ez);
            double exd = (double)ex, eyd = (double)ey, ezd = (double)ez;
            double Eg = sqrt(exd * exd + eyd * eyd + ezd * ezd) * 1e-9;
            bool cand = false;
            if (Eg > a.ebsi) {
                bsi++;
            } else if (Eg > a.fi_thr) {
                double pdt = a.adk_c * pow(20.5 * a.x32 / Eg, a.adk_e) * exp(-6.83 * a.x32 / Eg) * a.dt_fs;
                Draw2 u = draw2(a.seed, id, a.step, kTagFi, 0);
                uint32_t nc = (pdt > u.a) ? 1u : 0u;
                // every unit of a weighted neutral draws for itself (Sec. 2.3.2)
                const uint32_t wn = a.s.w ? a.s.w[i] : 1u;
                for (uint32_t q = 1; q < wn; ++q)
                    nc += (pdt > draw2(a.seed, id, a.step, kTagFi + kTagSub, q).a) ? 1u : 0u;
                cand = nc > 0;
                if (cand && a.fi_cnt) a.fi_cnt[i] = nc;
            }
            unsigned long long p = wave_append(&a.st->n_fi, cand);
            if (cand) a.fi_list[p] = (uint32_t)i;
        }
    }
    // per-block partials (largest speed, removals per boundary, neutrals
    // above the barrier-suppression field), reduced by k_push_final in block
    // order: no device-wide atomics on shared counters
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        unsigned int v = __shfl_xor(smax, o, 64);
        smax = v > smax ? v : smax;
    }
    __shared__ unsigned int shm[kBlock / 64];
    __shared__ unsigned int sh[kBlock / 64];
    if (lane_id() == 0) shm[threadIdx.x >> 6] = smax;
    unsigned int tl[5];
#pragma unroll
    for (int k = 1; k < 5; ++k) tl[k] = block_sum(lost[k], sh);
    unsigned int tb = block_sum(bsi, sh);  // the block reductions synchronize, shm is complete
    if (threadIdx.x == 0) {
        unsigned int m = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = shm[w] > m ? shm[w] : m;
        uint32_t* q = a.part + (int64_t)blockIdx.x * 8;
        q[0] = m;
        for (int k = 1; k < 5; ++k) q[k] = tl[k];
        q[5] = tb;
    }
    if ((SP == PIC_ION && MOVE) || (SP != PIC_NEUTRAL && MOVE && a.field0)) {
        __shared__ double shd[kBlock / 64];
        const double b0 = block_sum(bomb[0], shd);
        __syncthreads();
        const double b1 = block_sum(bomb[1], shd);
        __syncthreads();
        const double s0 = block_sum(sr, shd);
        if (threadIdx.x == 0) {
            double* q = a.dpart + (int64_t)blockIdx.x * 4;
            q[0] = b0;
            q[1] = b1;
            q[2] = s0;
        }
    }
}

// Reduction of the push partials of one species (one block of 1024
// threads; each thread loads up to 8 blocks' entries together: integer sums
// and a maximum, so the order does not matter).
constexpr int kFinalBlock = 1024;

// With dpart (moving ions, or charges with the circuit): the FP64 partials,
// each thread adding its blocks in order, then a fixed-order block sum:
// bomb_scale = m / 2 (h/dt)^2 turns sum |V|^2 into joules, sr_scale = q h/dt
// turns sum V . E0 into amperes.
template <int SP>
__global__ __launch_bounds__(kFinalBlock) void k_push_final(DevState* st, const uint32_t* part, int nblocks,
                                                            const double* dpart, double bomb_scale, double sr_scale) {
    __shared__ unsigned long long sh[kFinalBlock / 64];
    __shared__ unsigned int shm[kFinalBlock / 64];
    unsigned int m = 0;
    unsigned long long s[6] = {0, 0, 0, 0, 0, 0};
    for (int b0 = 0; b0 < nblocks; b0 += 8 * kFinalBlock) {
        uint4 lo[8];
        uint2 hi[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int b = b0 + u * kFinalBlock + (int)threadIdx.x;
            const uint32_t* q = part + (int64_t)(b < nblocks ? b : 0) * 8;
            lo[u] = *(const uint4*)q;
            hi[u] = *(const uint2*)(q + 4);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (b0 + u * kFinalBlock + (int)threadIdx.x >= nblocks) continue;
            m = lo[u].x > m ? lo[u].x : m;
            s[1] += lo[u].y;
            s[2] += lo[u].z;
            s[3] += lo[u].w;
            s[4] += hi[u].x;
            s[5] += hi[u].y;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        unsigned int v = __shfl_xor(m, o, 64);
        m = v > m ? v : m;
    }
    if (lane_id() == 0) shm[threadIdx.x >> 6] = m;
    unsigned long long t[6];
    for (int k = 1; k < 6; ++k) t[k] = block_sum(s[k], sh);
    if (threadIdx.x == 0) {
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = shm[w] > m ? shm[w] : m;
        if (m > st->smax_bits[SP]) st->smax_bits[SP] = m;
        for (int k = 1; k < 5; ++k) st->absorbed[SP][k] += t[k];
        st->bsi_count += t[5];
    }
    if (dpart) {
        __shared__ double shd[kFinalBlock / 64];
        double d[3] = {0.0, 0.0, 0.0};
        for (int b = (int)threadIdx.x; b < nblocks; b += kFinalBlock)
            for (int k = 0; k < 3; ++k) d[k] += dpart[(int64_t)b * 4 + k];
        double r[3];
        for (int k = 0; k < 3; ++k) {
            r[k] = block_sum(d[k], shd);
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (SP == PIC_ION) {
                st->bomb_e[0] += bomb_scale * r[0];
                st->bomb_e[1] += bomb_scale * r[1];
            }
            if (SP != PIC_NEUTRAL) st->isr[SP] = sr_scale * r[2];
        }
    }
}

// One step of the RC circuit (Sec. 2.3.1), explicit in time: I_tot = (V0 -
// V_gap) / R, V_gap += dt / C (I_tot - I_gap) with I_gap the Shockley-Ramo
// current of this step's push. The next solves hold the anode at V_gap.
__global__ void k_circuit(DevState* st, double V0, double R, double C, double dt) {
    const double ig = st->isr[0] + st->isr[1];
    const double it = (V0 - st->v_gap) / R;
    st->i_gap = ig;
    st->i_tot = it;
    st->v_gap = st->v_gap + dt / C * (it - ig);
}

// ---------------------------------------------------------------------------
// Charge deposit, the source of Eq. poi: CIC weights of x^{n+1} quantized per
// axis to 2^-13, 2^-13 and 2^-14, so every product is an integer number of
// 2^-40 e and the eight corners of a particle sum to 2^40 exactly. One
// workgroup per tile of 8^3 cells reads the tile's particles from the cell
// bins, accumulates the (8+1)^3 nodes of the tile in LDS with 64-bit LDS
// atomics, then adds each touched node to global memory with one atomic.
// Integer sums do not depend on order, so the result is deterministic.

template <typename T>
struct DepositArgs {
    Species<T> e, ion;
    const uint32_t* off;
    const uint2* bins;
    int64_t* rho;
    Grid g;
    DevState* st;
};

// A node takes charge only from the particles of the (at most 8) cells
// around it, which lie in at most 8 tiles; each particle adds at most 2^40
// units. With fewer than 2^20 particles per tile every node sum stays below
// 8 * 2^20 * 2^40 = 2^63, so a tile at or above that count is reported as a
// possible fixed-point overflow (sticky PIC_E_OVERFLOW).
constexpr uint32_t kTileOverflow = 1u << 20;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_deposit_tiles(DepositArgs<T> a) {
    constexpr int N1 = kTile + 1;
    __shared__ unsigned long long q[N1 * N1 * N1];
    const Grid& g = a.g;
    uint32_t tile = blockIdx.x;
    uint32_t b0 = a.off[(int64_t)tile * kTileCells], b1 = a.off[(int64_t)(tile + 1) * kTileCells];
    if (b0 == b1) return;
    if (b1 - b0 >= kTileOverflow) {
        if (threadIdx.x == 0) atomicCAS(&a.st->error, 0, PIC_E_OVERFLOW);
        return;
    }
    int tx = (int)(tile % g.ntx), ty = (int)((tile / g.ntx) % g.nty), tz = (int)(tile / (g.ntx * g.nty));
    int ox = tx * kTile, oy = ty * kTile, oz = tz * kTile;
    for (int m = threadIdx.x; m < N1 * N1 * N1; m += blockDim.x) q[m] = 0ull;
    __syncthreads();
    for (uint32_t b = b0 + threadIdx.x; b < b1; b += blockDim.x) {
        uint32_t e = a.bins[b].x;
        uint32_t s = e >> 30;
        if (s == PIC_NEUTRAL) continue;
        uint32_t i = e & 0x3FFFFFFFu;
        const Species<T>& P = s == PIC_ELECTRON ? a.e : a.ion;
        double X = (double)P.x[i], Y = (double)P.y[i], Z = (double)P.z[i];
        int ci = clampi((int)floor(X), 0, g.nx - 2), cj = clampi((int)floor(Y), 0, g.ny - 2),
            ck = clampi((int)floor(Z), 0, g.nz - 2);
        int64_t qx = quantize(X - ci, 13), qy = quantize(Y - cj, 13), qz = quantize(Z - ck, 14);
        // a superparticle of weight w carries w charges
        int64_t sg = (s == PIC_ELECTRON ? -1 : 1) * (P.w ? (int64_t)P.w[i] : 1);
        int64_t w[2][3] = {{8192 - qx, 8192 - qy, 16384 - qz}, {qx, qy, qz}};
        int lx = ci - ox, ly = cj - oy, lz = ck - oz;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            int dx = t & 1, dy = (t >> 1) & 1, dz = (t >> 2) & 1;
            int64_t v = sg * w[dx][0] * w[dy][1] * w[dz][2];
            atomicAdd(&q[((lz + dz) * N1 + (ly + dy)) * N1 + (lx + dx)], (unsigned long long)v);
        }
    }
    __syncthreads();
    unsigned long long* rho = (unsigned long long*)a.rho;
    for (int m = threadIdx.x; m < N1 * N1 * N1; m += blockDim.x) {
        unsigned long long v = q[m];
        if (v == 0ull) continue;
        int lx = m % N1, ly = (m / N1) % N1, lz = m / (N1 * N1);
        int i = ox + lx, j = oy + ly, k = oz + lz;
        if (i >= g.nx || j >= g.ny || k >= g.nz) continue;
        atomicAdd(rho + ((int64_t)k * g.ny + j) * g.nx + i, v);
    }
}

// ---------------------------------------------------------------------------
// Monte Carlo collisions (Sec. 2.2, Eqs. colp, du, newv; Table colls).
// Per cell and pair class -- (e, Cu) with elastic scattering and impact
// ionization, then (Cu+, Cu) with charge exchange -- the species with fewer
// particles in the cell is the projectile (tie: the charged one); projectiles
// in ascending id order take targets in ascending id order, cyclically
// shifted by floor(U_c N_t) with U_c drawn per cell, so no target is used
// twice; n is the target count over the cell volume. A pair collides when
// U1 < P = 1 - exp(-u n sigma_tot dt); U2 picks the process in proportion to
// its cross section. A particle has at most one event per step: a neutral
// with an (e, Cu) event keeps its place in the (Cu+, Cu) pairing but its pair
// is void. Null-collision test: with u bounded by the sum of the largest
// speeds of the two species and sigma_tot by the table maximum, U1 >= P_null
// rules out a collision before any velocity is read.

template <typename T>
struct MccArgs {
    Species<T> sp[3];
    Grid g;
    const uint32_t* off;
    uint2* bins;
    int64_t nc;  // number of cell keys
    uint32_t* big;
    uint32_t* mcc_list;   // small cells for the full collision pass, one segment per scanning wavefront
    uint32_t* mcc_count;  // cells in each wavefront's segment (then their exclusive prefix sums)
    uint32_t* mcc_dense;  // the listed cells of all segments, in segment order
    const uint32_t* mcc_total;  // number of listed cells
    DevState* st;
    uint32_t step;
    uint64_t seed;
    double h, dt, m_ion, xi;
    const double* xs;   // el, iz, cx tables, then the rate bounds of the two pair classes
    int xs_n;
    double xs_emin, xs_lnr;
    uint32_t* nflag;
    uint32_t* bitmap_imp;
    uint32_t* prod_list;
    double* prod_ve;
    int32_t* prod_ev;
    pic_event* ev;
    int64_t ev_cap;
    int record, write_sorted;
    // superparticle weights (weighted runs only)
    int weighted;
    uint32_t* prod_c;         // per neutral slot: ionized units of its product
    uint32_t* fi_cnt;         // per neutral slot: field-ionized units (from the push)
    uint32_t* split_list[3];  // per species: parent slots of the split-offs
    uint32_t* split_c[3];     // per species and slot: units split off
    double* split_v[3];       // per species and slot: their velocity
    uint32_t* split_bm[3];    // per species: parents as a bitmap over ids
};

// The c collided units of superparticle p of species sp take the velocity
// v (grid units): in place when they are the whole superparticle, else they
// are split off (Sec. 2.3.2) as a new superparticle made in the products
// phase in the order (species, parent id); the parent keeps the rest and its
// velocity.
template <typename T>
__device__ inline void collided_units(const MccArgs<T>& a, const Species<T>& S, int sp, uint32_t p, const double v[3],
                                      uint32_t c) {
    const uint32_t w = S.w ? S.w[p] : 1u;
    if (c >= w) {
        S.vx[p] = (T)v[0];
        S.vy[p] = (T)v[1];
        S.vz[p] = (T)v[2];
        return;
    }
    const unsigned long long q = atomicAdd(&a.st->n_split[sp], 1ull);
    a.split_list[sp][q] = p;
    a.split_c[sp][p] = c;
    a.split_v[sp][3 * (int64_t)p + 0] = v[0];
    a.split_v[sp][3 * (int64_t)p + 1] = v[1];
    a.split_v[sp][3 * (int64_t)p + 2] = v[2];
    const uint32_t id = S.id[p];
    atomicOr(&a.split_bm[sp][id >> 5], 1u << (id & 31));
}

// Linear index of the cell with this key: the per-cell draw is keyed by it.
__device__ inline uint32_t linear_cell(const Grid& g, uint32_t key) {
    int i, j, k;
    key_cell(g, key, i, j, k);
    return (uint32_t)(((int64_t)k * (g.ny - 1) + j) * (g.nx - 1) + i);
}

__device__ inline double xs_lookup(const double* tab, int n, double emin, double lnr, double E) {
    if (E <= emin) return tab[0];
    double emax = emin * exp(lnr);
    if (E >= emax) return tab[n - 1];
    double t = log(E / emin) / lnr * (double)(n - 1);
    int k = (int)floor(t);
    k = k > n - 2 ? n - 2 : (k < 0 ? 0 : k);
    double f = t - k;
    return tab[k] + f * (tab[k + 1] - tab[k]);
}

__device__ inline void iso_dir(double ct, double ph, double s[3]) {
    double st = sqrt(1.0 - ct * ct);
    double sp, cp;
    sincos(ph, &sp, &cp);
    s[0] = st * cp;
    s[1] = st * sp;
    s[2] = ct;
}

template <typename T>
__device__ inline int64_t record_event(const MccArgs<T>& a, int kind, uint32_t ida, uint32_t idb) {
    if (!a.record) return -1;
    unsigned long long p = atomicAdd(&a.st->n_ev, 1ull);
    if ((int64_t)p >= a.ev_cap) return -1;
    pic_event e;
    e.kind = kind;
    e.id_a = ida;
    e.id_b = idb;
    e.new_ion = kDead;
    e.new_e = kDead;
    a.ev[p] = e;
    return (int64_t)p;
}

// Decide and apply one pair of class cls (1: e-Cu, 2: Cu+-Cu). ia indexes the
// charged particle, ib the neutral; pid is the projectile id. Returns the
// event kind, or 0; nc receives N_coll, the collided units (Sec. 2.3.2: the
// lighter superparticle is cut into min(w_a, w_b) sub-particles, each
// colliding with the heavier one with P = 1 - exp(-u n w_t sigma dt); with
// every weight 1 this is one binary collision).
template <typename T>
__device__ int resolve_pair(const MccArgs<T>& a, int cls, uint32_t pid, uint32_t ia, uint32_t ib, int NT,
                            double pnull, uint32_t& nc) {
    const uint32_t tag = cls == 1 ? kTagMcc1 : kTagMcc2;
    Draw2 d = draw2(a.seed, pid, a.step, tag, 0);
    if (d.a >= pnull) return 0;  // null collision (pnull is 2 in weighted runs)
    const Species<T>& A = a.sp[cls == 1 ? PIC_ELECTRON : PIC_ION];
    const Species<T>& B = a.sp[PIC_NEUTRAL];
    const uint32_t wa = A.w ? A.w[ia] : 1u, wb = B.w ? B.w[ib] : 1u;
    const uint32_t wt = wa > wb ? wa : wb, npart = wa < wb ? wa : wb;
    double s = a.h / a.dt;
    double vA[3] = {(double)A.vx[ia], (double)A.vy[ia], (double)A.vz[ia]};
    double vB[3] = {(double)B.vx[ib], (double)B.vy[ib], (double)B.vz[ib]};
    double u[3] = {(vA[0] - vB[0]) * s, (vA[1] - vB[1]) * s, (vA[2] - vB[2]) * s};
    double um = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    double mA = cls == 1 ? kMe : a.m_ion;
    double E = 0.5 * mA * um * um / kQe;
    double sig0, sig1 = 0.0;
    if (cls == 1) {
        sig0 = xs_lookup(a.xs, a.xs_n, a.xs_emin, a.xs_lnr, E);
        sig1 = (E > a.xi) ? xs_lookup(a.xs + a.xs_n, a.xs_n, a.xs_emin, a.xs_lnr, E) : 0.0;
    } else {
        sig0 = xs_lookup(a.xs + 2 * a.xs_n, a.xs_n, a.xs_emin, a.xs_lnr, E);
    }
    double stot = sig0 + sig1;
    double n = (double)NT / (a.h * a.h * a.h);
    double P = -expm1(-um * n * (double)wt * stot * a.dt);
    uint32_t ncoll = (d.a < P) ? 1u : 0u;
    for (uint32_t q = 1; q < npart; ++q) ncoll += (draw2(a.seed, pid, a.step, tag + kTagSub, q).a < P) ? 1u : 0u;
    nc = ncoll;
    if (ncoll == 0) return 0;
    uint32_t idA = A.id[ia], idB = B.id[ib];
    if (cls == 2) {
        // charge exchange: the collided units exchange their velocities
        const double na[3] = {vB[0], vB[1], vB[2]}, nb[3] = {vA[0], vA[1], vA[2]};
        collided_units(a, A, PIC_ION, ia, na, ncoll);
        collided_units(a, B, PIC_NEUTRAL, ib, nb, ncoll);
        record_event(a, PIC_EV_CX, idA, idB);
        return PIC_EV_CX;
    }
    bool elastic = d.b * stot < sig0;
    double g = a.dt / a.h;
    if (elastic) {
        // Eq. du: Delta u = R^-1(theta, phi) [R^-1(theta', phi') - I] (0,0,u),
        // (theta, phi) the direction of u, (theta', phi') isotropic; Eq. newv.
        Draw2 r = draw2(a.seed, pid, a.step, kTagMcc1, 1);
        double ct2 = 2.0 * r.a - 1.0, ph2 = 2.0 * kPi * r.b;
        double up = sqrt(u[0] * u[0] + u[1] * u[1]);
        double ct = u[2] / um, st = up / um, cp = 1.0, sp = 0.0;
        if (up > 0.0) {
            cp = u[0] / up;
            sp = u[1] / up;
        }
        double st2 = sqrt(1.0 - ct2 * ct2);
        double sp2, cp2;
        sincos(ph2, &sp2, &cp2);
        double w0 = um * st2 * cp2, w1 = um * st2 * sp2, w2 = um * (ct2 - 1.0);
        double du0 = ct * cp * w0 - sp * w1 + st * cp * w2;
        double du1 = ct * sp * w0 + cp * w1 + st * sp * w2;
        double du2 = -st * w0 + ct * w2;
        double mu = mA * a.m_ion / (mA + a.m_ion);
        double ka = mu / mA * g, kb = mu / a.m_ion * g;
        const double na[3] = {vA[0] + ka * du0, vA[1] + ka * du1, vA[2] + ka * du2};
        const double nb[3] = {vB[0] - kb * du0, vB[1] - kb * du1, vB[2] - kb * du2};
        collided_units(a, A, PIC_ELECTRON, ia, na, ncoll);
        collided_units(a, B, PIC_NEUTRAL, ib, nb, ncoll);
        record_event(a, PIC_EV_ELASTIC, idA, idB);
        return PIC_EV_ELASTIC;
    }
    // Impact ionization Cu + e -> Cu+ + 2e: in the rest frame of the neutral
    // the energy above xi is shared as U5 : 1 - U5 by the scattered and the
    // new electron, both leaving isotropically; the ion keeps the neutral's
    // position and velocity, the new electron starts at that position. The
    // ion and the new electron carry the ionized units, which the neutral
    // loses in the products phase.
    Draw2 r1 = draw2(a.seed, pid, a.step, kTagMcc1, 1);
    Draw2 r2 = draw2(a.seed, pid, a.step, kTagMcc1, 2);
    Draw2 r3 = draw2(a.seed, pid, a.step, kTagMcc1, 3);
    double s1[3], s2[3];
    iso_dir(2.0 * r1.a - 1.0, 2.0 * kPi * r1.b, s1);
    iso_dir(2.0 * r2.a - 1.0, 2.0 * kPi * r2.b, s2);
    double erem = E - a.xi;
    double e1 = r3.a * erem, e2 = erem - e1;
    double w1 = sqrt(2.0 * e1 * kQe / kMe), w2 = sqrt(2.0 * e2 * kQe / kMe);
    double vn[3] = {vB[0] * s, vB[1] * s, vB[2] * s};
    const double v1[3] = {(vn[0] + w1 * s1[0]) * g, (vn[1] + w1 * s1[1]) * g, (vn[2] + w1 * s1[2]) * g};
    collided_units(a, A, PIC_ELECTRON, ia, v1, ncoll);
    a.prod_ve[3 * (int64_t)ib + 0] = (vn[0] + w2 * s2[0]) * g;
    a.prod_ve[3 * (int64_t)ib + 1] = (vn[1] + w2 * s2[1]) * g;
    a.prod_ve[3 * (int64_t)ib + 2] = (vn[2] + w2 * s2[2]) * g;
    if (a.prod_c) a.prod_c[ib] = ncoll;
    atomicOr(&a.bitmap_imp[idB >> 5], 1u << (idB & 31));
    unsigned long long p = wave_append(&a.st->n_prod, true);
    a.prod_list[p] = ib;  // kind 0 (impact); n_prod_kind[0] is added per block
    a.prod_ev[ib] = (int32_t)record_event(a, PIC_EV_IONIZE, idA, idB);
    return PIC_EV_IONIZE;
}

// P_null of class cls for NT targets: an upper bound of the collision
// probability of every pair of the class this step, from the largest
// relative speed U (the largest speeds of the two species, rounded up) and
// the bound of u sigma_tot(E(u)) over u <= U (the table entry one segment
// above that of E(U), against rounding in the index; above the last node
// sigma is the last value).
template <typename T>
__device__ inline double pnull_of(const MccArgs<T>& a, int cls, int NT) {
    // weighted pairs collide with more than one draw and a weighted target
    // probability: no null-collision bound, every pair is decided in full
    if (a.weighted) return 2.0;
    const int sa = cls == 1 ? PIC_ELECTRON : PIC_ION;
    const double ug = ((double)__uint_as_float(a.st->smax_bits[sa]) + (double)__uint_as_float(a.st->smax_bits[2])) *
                      (1.0 + 0x1p-20);
    const double U = ug * a.h / a.dt;
    const double m = cls == 1 ? kMe : a.m_ion;
    const double E = 0.5 * m * U * U / kQe;
    const int n = a.xs_n;
    const double* nu = a.xs + (size_t)(2 + cls) * n;
    double rate;
    if (E >= a.xs_emin * exp(a.xs_lnr)) {
        const double slast = cls == 1 ? a.xs[n - 1] + a.xs[2 * n - 1] : a.xs[3 * n - 1];
        rate = fmax(nu[n - 1], U * slast);
    } else {
        int k = E <= a.xs_emin ? 0 : (int)floor(log(E / a.xs_emin) / a.xs_lnr * (double)(n - 1));
        k = k + 1 > n - 1 ? n - 1 : (k + 1 < 0 ? 0 : k + 1);
        rate = nu[k];
    }
    const double x = rate * (double)NT / (a.h * a.h * a.h) * a.dt * (1.0 + 1e-9);
    return -expm1(-x);
}

// Pairs of one class inside one cell, sequentially. Entries are sorted by
// (species, id); [a0, a0+na) charged species, [b0, b0+nb) neutrals.
// used: bit r set if the neutral of rank r had an event (input and output).
// pn: P_null of this class by target count (NT <= kSmallCell), or null to
// compute it.
template <typename T>
__device__ void cell_class_seq(const MccArgs<T>& a, int cls, uint32_t cell, const uint64_t* kk, const uint32_t* ee,
                               int a0, int na, int b0, int nb, uint32_t& used, int cnt[10], const double* pn = nullptr) {
    if (na == 0 || nb == 0) return;
    bool a_proj = na <= nb;
    int P0 = a_proj ? a0 : b0, NP = a_proj ? na : nb;
    int T0 = a_proj ? b0 : a0, NT = a_proj ? nb : na;
    // the pairing shift (a single target needs no draw: the shift is 0)
    int shift = 0;
    if (NT > 1) {
        Draw2 dc = draw2(a.seed, linear_cell(a.g, cell), a.step, cls == 1 ? kTagPair1 : kTagPair2, 0);
        shift = (int)floor(dc.a * (double)NT);
        shift = shift > NT - 1 ? NT - 1 : shift;
    }
    double pnull = pn ? pn[NT] : pnull_of(a, cls, NT);
    for (int i = 0; i < NP; ++i) {
        int pi = P0 + i, ti = T0 + (shift + i) % NT;
        int ai = a_proj ? pi : ti, bi = a_proj ? ti : pi;
        int brank = bi - b0;
        if (cls == 2 && ((used >> brank) & 1u)) continue;
        uint32_t pid = (uint32_t)(kk[pi] & 0xFFFFFFFFu);
        uint32_t nc = 0;
        int kind = resolve_pair(a, cls, pid, ee[ai] & 0x3FFFFFFFu, ee[bi] & 0x3FFFFFFFu, NT, pnull, nc);
        if (kind) {
            used |= 1u << brank;
            a.nflag[ee[bi] & 0x3FFFFFFFu] = a.step + 1u;
            cnt[kind]++;
            cnt[5 + kind] += (int)nc;
        }
    }
}

template <typename T>
__device__ inline void flush_counts(DevState* st, int cnt[10]) {
    __shared__ int sh[kBlock / 64];
    for (int k = 1; k <= 3; ++k) {
        int t = block_sum(cnt[k], sh);
        if (threadIdx.x == 0 && t) {
            atomicAdd(&st->events[k], (unsigned long long)t);
            if (k == PIC_EV_IONIZE) atomicAdd(&st->n_prod_kind[0], (unsigned long long)t);
        }
        int tw = block_sum(cnt[5 + k], sh);
        if (threadIdx.x == 0 && tw) atomicAdd(&st->events_w[k], (unsigned long long)tw);
    }
}

// Collisions of one cell of 2 .. kSmallCell particles (one lane).
template <typename T>
__device__ inline void mcc_cell(const MccArgs<T>& a, uint32_t c, uint32_t o0, int n, const double (*pn)[kSmallCell + 1],
                                int cnt[10]) {
    uint64_t kk[kSmallCell];
    uint32_t ee[kSmallCell];
    for (int t = 0; t < n; ++t) {
        const uint2 be = a.bins[o0 + t];
        uint32_t e = be.x;
        uint32_t s = e >> 30;
        uint64_t k = ((uint64_t)s << 32) | be.y;
        int u = t;
        while (u > 0 && kk[u - 1] > k) {
            kk[u] = kk[u - 1];
            ee[u] = ee[u - 1];
            --u;
        }
        kk[u] = k;
        ee[u] = e;
    }
    if (a.write_sorted)
        for (int t = 0; t < n; ++t) a.bins[o0 + t] = make_uint2(ee[t], (uint32_t)kk[t]);
    int ne = 0, ni = 0;
    for (int t = 0; t < n; ++t) {
        uint32_t s = (uint32_t)(kk[t] >> 32);
        ne += s == 0;
        ni += s == 1;
    }
    int nn = n - ne - ni;
    uint32_t used = 0;
    cell_class_seq(a, 1, c, kk, ee, 0, ne, ne + ni, nn, used, cnt, pn[0]);
    cell_class_seq(a, 2, c, kk, ee, ne, ni, ne + ni, nn, used, cnt, pn[1]);
}

// Whether a cell of 2 .. kSmallCell particles can have a collision: some
// projectile of class 1 or 2 draws below P_null. The null-collision draw of a
// projectile depends only on its id, the step and the class (not on the
// pairing), so a cell where every projectile draws a null collision has no
// event and leaves every state unchanged (the full pass would skip each of
// its pairs); the test ignores the neutrals already used by class 1, so it
// may list a cell that then has no event, never the reverse.
template <typename T>
__device__ inline bool mcc_probe(const MccArgs<T>& a, uint32_t o0, int n, const double (*pn)[kSmallCell + 1]) {
    uint32_t e[kSmallCell], id[kSmallCell];
#pragma unroll
    for (int t = 0; t < kSmallCell; ++t) {
        const uint2 be = a.bins[o0 + (t < n ? t : 0)];
        e[t] = be.x;
        id[t] = be.y;
    }
    int cs[3] = {0, 0, 0};
#pragma unroll
    for (int t = 0; t < kSmallCell; ++t) {
        const uint32_t sp = e[t] >> 30;
        if (t < n) cs[sp] += 1;
    }
    // projectiles of each class as bit masks over the cell's entries
    uint32_t pm[2] = {0u, 0u};
    double pnull[2] = {0.0, 0.0};
#pragma unroll
    for (int cls = 1; cls <= 2; ++cls) {
        const int na = cs[cls - 1], nb = cs[2];
        if (na == 0 || nb == 0) continue;
        const bool a_proj = na <= nb;
        const uint32_t psp = a_proj ? (uint32_t)(cls - 1) : 2u;
        pnull[cls - 1] = pn[cls - 1][a_proj ? nb : na];
#pragma unroll
        for (int t = 0; t < kSmallCell; ++t)
            if (t < n && (e[t] >> 30) == psp) pm[cls - 1] |= 1u << t;
    }
    // one draw per projectile (class 1 first), until one is below P_null
#pragma unroll 1
    while (pm[0] | pm[1]) {
        const int cls = pm[0] ? 1 : 2;
        const int t = __ffs(cls == 1 ? pm[0] : pm[1]) - 1;
        if (cls == 1)
            pm[0] &= pm[0] - 1u;
        else
            pm[1] &= pm[1] - 1u;
        uint32_t pid = id[0];
#pragma unroll
        for (int u = 1; u < kSmallCell; ++u) pid = t == u ? id[u] : pid;
        const Draw2 d = draw2(a.seed, pid, a.step, cls == 1 ? kTagMcc1 : kTagMcc2, 0);
        if (d.a < (cls == 1 ? pnull[0] : pnull[1])) return true;
    }
    return false;
}

// P_null by class and target count (the same in every block)
template <typename T>
__device__ inline void pnull_table(const MccArgs<T>& a, double (*pn)[kSmallCell + 1]) {
    if (threadIdx.x < 2 * (kSmallCell + 1)) {
        const int cls = 1 + (int)threadIdx.x / (kSmallCell + 1), nt = (int)threadIdx.x % (kSmallCell + 1);
        pn[cls - 1][nt] = nt > 0 ? pnull_of(a, cls, nt) : 0.0;
    }
    __syncthreads();
}

// The range of cells of scanning wavefront gw of nw: [cb, ce).
__device__ inline void mcc_range(int64_t nc, int64_t nw, int64_t gw, int64_t& cb, int64_t& ce) {
    const int64_t per = ((nc + nw - 1) / nw + 63) / 64 * 64;
    cb = gw * per;
    ce = cb + per < nc ? cb + per : nc;
}

// Cells with 2 .. kSmallCell particles: each wavefront scans its own range
// of cells 64 at a time and gathers the cells with 2 .. kSmallCell particles
// in a queue in LDS (ballot and prefix count; most cells hold fewer than
// two), then tests 64 of them at once with every lane busy, and lists those
// that can have a collision (all of them when the sorted order is to be
// written back) in its own segment of the list (the part of the list from
// the first cell of its range on; no counter shared between wavefronts).
// Larger cells are listed for k_mcc_big: up to kMidCell particles from the
// start of the list, more from its end.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_mcc_small(MccArgs<T> a) {
    __shared__ double pn[2][kSmallCell + 1];
    __shared__ uint32_t queue[kBlock / 64][128];
    pnull_table(a, pn);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t* q = queue[w];
    const int64_t nw = (int64_t)gridDim.x * (kBlock / 64);
    const int64_t gw = (int64_t)blockIdx.x * (kBlock / 64) + w;
    int64_t cb, ce;
    mcc_range(a.nc, nw, gw, cb, ce);
    int qn = 0;        // the same in every lane
    uint32_t nl = 0;   // cells listed so far (the same in every lane)
    int64_t c0 = cb;
    while (c0 < ce || qn > 0) {
        while (qn < 64 && c0 < ce) {
            const int64_t c = c0 + lane;
            int n = 0;
            uint32_t o0 = 0;
            if (c < ce) {
                o0 = a.off[c];
                n = (int)(a.off[c + 1] - o0);
            }
            if (n > kSmallCell && n <= kMidCell) {
                unsigned long long p = atomicAdd(&a.st->n_big, 1ull);
                a.big[p] = (uint32_t)c;
            } else if (n > kMidCell) {
                // the larger cells from the end of the list
                unsigned long long p = atomicAdd(&a.st->n_big2, 1ull);
                a.big[a.nc - 1 - (int64_t)p] = (uint32_t)c;
            }
            const bool act = n >= 2 && n <= kSmallCell;
            const unsigned long long m = __ballot(act);
            if (act) q[qn + __popcll(m & ((1ull << lane) - 1ull))] = (uint32_t)c;
            qn += __popcll(m);
            c0 += 64;
        }
        __builtin_amdgcn_wave_barrier();
        const int take = qn < 64 ? qn : 64;
        uint32_t c = 0;
        bool full = false;
        if (lane < take) {
            c = q[lane];
            const uint32_t o0 = a.off[c];
            full = a.write_sorted || mcc_probe(a, o0, (int)(a.off[c + 1] - o0), pn);
        }
        const unsigned long long fm = __ballot(full);
        if (full) a.mcc_list[cb + nl + __popcll(fm & ((1ull << lane) - 1ull))] = c;
        nl += (uint32_t)__popcll(fm);
        // move the cells not taken to the front of the queue
        const int rest = qn - take;
        const uint32_t keep = lane < rest ? q[take + lane] : 0u;
        __builtin_amdgcn_wave_barrier();
        if (lane < rest) q[lane] = keep;
        __builtin_amdgcn_wave_barrier();
        qn = rest;
    }
    if (lane == 0 && gw < nw) a.mcc_count[gw] = nl;
}

// The segments of k_mcc_small (launched with the same grid) copied one
// after another into mcc_dense: wavefront gw copies its segment to the
// prefix sum of the counts before it.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_mcc_compact(MccArgs<T> a) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t nw = (int64_t)gridDim.x * (kBlock / 64);
    const int64_t gw = (int64_t)blockIdx.x * (kBlock / 64) + w;
    int64_t cb, ce;
    mcc_range(a.nc, nw, gw, cb, ce);
    const uint32_t o = a.mcc_count[gw];
    const uint32_t nl = (gw + 1 < nw ? a.mcc_count[gw + 1] : *a.mcc_total) - o;
    for (uint32_t t = (uint32_t)lane; t < nl; t += 64) a.mcc_dense[o + t] = a.mcc_list[cb + t];
}

// Collisions of the listed cells, one lane per cell (every lane of a
// wavefront busy but in the last one).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_mcc_cells(MccArgs<T> a) {
    __shared__ double pn[2][kSmallCell + 1];
    pnull_table(a, pn);
    int cnt[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t nl = (int64_t)*a.mcc_total;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nl; t += stride) {
        const uint32_t c = a.mcc_dense[t];
        const uint32_t o0 = a.off[c];
        mcc_cell(a, c, o0, (int)(a.off[c + 1] - o0), pn, cnt);
    }
    flush_counts<T>(a.st, cnt);
}

// One wavefront per cell with more than kSmallCell particles: bitonic sort of
// the (species, id) keys in LDS, then projectiles handled across the lanes.
// CAP = kMidCell takes the cells listed from the start of the list (small
// LDS arrays, so that many wavefronts share a compute unit), CAP = kBigCell
// those from its end up to kBigCell particles.
template <typename T, int CAP>
__global__ __launch_bounds__(64) void k_mcc_big(MccArgs<T> a) {
    __shared__ uint64_t kk[CAP];
    __shared__ uint32_t ee[CAP];
    __shared__ uint8_t used[CAP];
    constexpr bool kBack = CAP > kMidCell;
    int cnt[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int lane = threadIdx.x;
    const int64_t nbig = (int64_t)(kBack ? a.st->n_big2 : a.st->n_big);
    for (int64_t b = blockIdx.x; b < nbig; b += gridDim.x) {
        uint32_t c = kBack ? a.big[a.nc - 1 - b] : a.big[b];
        uint32_t o0 = a.off[c];
        int n = (int)(a.off[c + 1] - o0);
        if (n > CAP) continue;  // k_mcc_huge
        int P = 1;
        while (P < n) P <<= 1;
        for (int t = lane; t < P; t += 64) {
            if (t < n) {
                const uint2 be = a.bins[o0 + t];
                uint32_t e = be.x;
                uint32_t s = e >> 30;
                kk[t] = ((uint64_t)s << 32) | be.y;
                ee[t] = e;
            } else {
                kk[t] = ~0ull;
                ee[t] = 0;
            }
            used[t] = 0;
        }
        __syncthreads();
        for (int k = 2; k <= P; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int t = lane; t < P; t += 64) {
                    int u = t ^ j;
                    if (u > t) {
                        bool up = (t & k) == 0;
                        uint64_t x = kk[t], y = kk[u];
                        if ((x > y) == up) {
                            kk[t] = y;
                            kk[u] = x;
                            uint32_t ex = ee[t];
                            ee[t] = ee[u];
                            ee[u] = ex;
                        }
                    }
                }
                __syncthreads();
            }
        }
        if (a.write_sorted)
            for (int t = lane; t < n; t += 64) a.bins[o0 + t] = make_uint2(ee[t], (uint32_t)kk[t]);
        int ne = 0, ni = 0;
        for (int t = lane; t < n; t += 64) {
            uint32_t s = (uint32_t)(kk[t] >> 32);
            ne += s == 0;
            ni += s == 1;
        }
        ne = wave_sum(ne);
        ni = wave_sum(ni);
        int nn = n - ne - ni;
        for (int cls = 1; cls <= 2; ++cls) {
            int a0 = cls == 1 ? 0 : ne, na = cls == 1 ? ne : ni, b0 = ne + ni, nb = nn;
            if (na > 0 && nb > 0) {
                bool a_proj = na <= nb;
                int P0 = a_proj ? a0 : b0, NP = a_proj ? na : nb;
                int T0 = a_proj ? b0 : a0, NT = a_proj ? nb : na;
                Draw2 dc = draw2(a.seed, linear_cell(a.g, c), a.step, cls == 1 ? kTagPair1 : kTagPair2, 0);
                int shift = (int)floor(dc.a * (double)NT);
                shift = shift > NT - 1 ? NT - 1 : shift;
                double pnull = pnull_of(a, cls, NT);
                for (int i = lane; i < NP; i += 64) {
                    int pi = P0 + i, ti = T0 + (shift + i) % NT;
                    int ai = a_proj ? pi : ti, bi = a_proj ? ti : pi;
                    if (cls == 2 && used[bi]) continue;
                    uint32_t pid = (uint32_t)(kk[pi] & 0xFFFFFFFFu);
                    uint32_t nc = 0;
                    int kind = resolve_pair(a, cls, pid, ee[ai] & 0x3FFFFFFFu, ee[bi] & 0x3FFFFFFFu, NT, pnull, nc);
                    if (kind) {
                        used[bi] = 1;
                        a.nflag[ee[bi] & 0x3FFFFFFFu] = a.step + 1u;
                        cnt[kind]++;
                        cnt[5 + kind] += (int)nc;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int k = 1; k <= 3; ++k) {
        int t = wave_sum(cnt[k]);
        if (lane == 0 && t) {
            atomicAdd(&a.st->events[k], (unsigned long long)t);
            if (k == PIC_EV_IONIZE) atomicAdd(&a.st->n_prod_kind[0], (unsigned long long)t);
        }
        int tw = wave_sum(cnt[5 + k]);
        if (lane == 0 && tw) atomicAdd(&a.st->events_w[k], (unsigned long long)tw);
    }
}

// Cells of more than kBigCell particles (a dense plasma near the tip): one
// block of kHugeThreads per cell. The cell's bin entries are sorted by
// (species, id) in place in global memory by a bitonic network whose
// comparators all put the smaller key first (each merge starts with the
// mirrored pairs), so the virtual +inf keys that pad the count to a power
// of two never move and are never stored; the pair classes then run as in
// k_mcc_big with the per-entry used flags in global memory (flags, indexed
// by bin position).
constexpr int kHugeThreads = 1024;

__device__ inline uint64_t bin_key(uint2 e) { return ((uint64_t)(e.x >> 30) << 32) | e.y; }

__device__ inline void huge_cmpx(uint2* e, int n, int i, int j) {
    if (j >= n) return;  // e[j] is +inf
    const uint2 x = e[i], y = e[j];
    if (bin_key(x) > bin_key(y)) {
        e[i] = y;
        e[j] = x;
    }
}

template <typename T>
__global__ __launch_bounds__(kHugeThreads) void k_mcc_huge(MccArgs<T> a, uint32_t* flags) {
    __shared__ int sh[kHugeThreads / 64];
    int cnt[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int tid = threadIdx.x;
    const int64_t nbig = (int64_t)a.st->n_big2;  // the larger cells, listed from the end
    for (int64_t b = blockIdx.x; b < nbig; b += gridDim.x) {
        const uint32_t c = a.big[a.nc - 1 - b];
        const uint32_t o0 = a.off[c];
        const int n = (int)(a.off[c + 1] - o0);
        if (n <= kBigCell) continue;
        uint2* e = a.bins + o0;
        uint32_t* used = flags + o0;
        int P = 1;
        while (P < n) P <<= 1;
        for (int k = 2; k <= P; k <<= 1) {
            const int hk = k >> 1;
            for (int t = tid; t < P / 2; t += kHugeThreads) {
                const int base = (t / hk) * k, r = t % hk;
                huge_cmpx(e, n, base + r, base + k - 1 - r);
            }
            __syncthreads();
            for (int j = k >> 2; j > 0; j >>= 1) {
                for (int t = tid; t < P / 2; t += kHugeThreads) {
                    const int i = (t / j) * 2 * j + t % j;
                    huge_cmpx(e, n, i, i + j);
                }
                __syncthreads();
            }
        }
        int ne = 0, ni = 0;
        for (int t = tid; t < n; t += kHugeThreads) {
            const uint32_t sp = e[t].x >> 30;
            ne += sp == 0;
            ni += sp == 1;
            used[t] = 0u;
        }
        ne = block_sum(ne, sh);
        if (tid == 0) sh[0] = ne;
        __syncthreads();
        ne = sh[0];
        __syncthreads();
        ni = block_sum(ni, sh);
        if (tid == 0) sh[0] = ni;
        __syncthreads();
        ni = sh[0];
        __syncthreads();
        const int nn = n - ne - ni;
        for (int cls = 1; cls <= 2; ++cls) {
            const int a0 = cls == 1 ? 0 : ne, na = cls == 1 ? ne : ni, b0 = ne + ni, nb = nn;
            if (na > 0 && nb > 0) {
                const bool a_proj = na <= nb;
                const int P0 = a_proj ? a0 : b0, NP = a_proj ? na : nb;
                const int T0 = a_proj ? b0 : a0, NT = a_proj ? nb : na;
                const Draw2 dc = draw2(a.seed, linear_cell(a.g, c), a.step, cls == 1 ? kTagPair1 : kTagPair2, 0);
                int shift = (int)floor(dc.a * (double)NT);
                shift = shift > NT - 1 ? NT - 1 : shift;
                const double pnull = pnull_of(a, cls, NT);
                for (int i = tid; i < NP; i += kHugeThreads) {
                    const int pi = P0 + i, ti = T0 + (shift + i) % NT;
                    const int ai = a_proj ? pi : ti, bi = a_proj ? ti : pi;
                    if (cls == 2 && used[bi]) continue;
                    const uint32_t pid = e[pi].y;
                    uint32_t nc = 0;
                    const int kind =
                        resolve_pair(a, cls, pid, e[ai].x & 0x3FFFFFFFu, e[bi].x & 0x3FFFFFFFu, NT, pnull, nc);
                    if (kind) {
                        used[bi] = 1u;
                        a.nflag[e[bi].x & 0x3FFFFFFFu] = a.step + 1u;
                        cnt[kind]++;
                        cnt[5 + kind] += (int)nc;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int k = 1; k <= 3; ++k) {
        const int t = block_sum(cnt[k], sh);
        if (tid == 0 && t) {
            atomicAdd(&a.st->events[k], (unsigned long long)t);
            if (k == PIC_EV_IONIZE) atomicAdd(&a.st->n_prod_kind[0], (unsigned long long)t);
        }
        const int tw = block_sum(cnt[5 + k], sh);
        if (tid == 0 && tw) atomicAdd(&a.st->events_w[k], (unsigned long long)tw);
    }
}

// Field ionization of the candidates whose neutral had no collision event.
template <typename T>
__global__ void k_fi_resolve(MccArgs<T> a, const uint32_t* fi_list, uint32_t* bitmap_fi) {
    int64_t n = (int64_t)a.st->n_fi;
    int cnt = 0, cntw = 0;
    const Species<T>& N = a.sp[PIC_NEUTRAL];
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint32_t ib = fi_list[i];
        bool go = a.nflag[ib] != a.step + 1u;
        unsigned long long p = wave_append(&a.st->n_prod, go);
        if (!go) continue;
        a.nflag[ib] = a.step + 1u;
        uint32_t id = N.id[ib];
        const uint32_t nc = a.fi_cnt ? a.fi_cnt[ib] : 1u;
        if (a.prod_c) a.prod_c[ib] = nc;
        cntw += (int)nc;
        atomicOr(&bitmap_fi[id >> 5], 1u << (id & 31));
        a.prod_ve[3 * (int64_t)ib + 0] = (double)N.vx[ib];
        a.prod_ve[3 * (int64_t)ib + 1] = (double)N.vy[ib];
        a.prod_ve[3 * (int64_t)ib + 2] = (double)N.vz[ib];
        a.prod_list[p] = ib | 0x80000000u;
        a.prod_ev[ib] = (int32_t)record_event(a, PIC_EV_FIELD_ION, kDead, id);
        ++cnt;
    }
    __shared__ int sh[kBlock / 64];
    int t = block_sum(cnt, sh);
    if (threadIdx.x == 0 && t) {
        atomicAdd(&a.st->events[PIC_EV_FIELD_ION], (unsigned long long)t);
        atomicAdd(&a.st->n_prod_kind[1], (unsigned long long)t);
    }
    int tw = block_sum(cntw, sh);
    if (threadIdx.x == 0 && tw) atomicAdd(&a.st->events_w[PIC_EV_FIELD_ION], (unsigned long long)tw);
}

// ---------------------------------------------------------------------------
// Products of ionization. They are numbered in the order (impact before
// field ionization, ascending neutral id): the rank of a product is the
// number of products before it in that order, read from per-kind bitmaps over
// the id space and their word prefix counts. Each product takes the ids
// next_id + 2 rank (ion) and next_id + 2 rank + 1 (electron) and the slots
// n_slots + rank of the ion and electron arrays; the neutral's slot is freed.

template <typename T>
struct ProdArgs {
    Species<T> sp[3];
    DevState* st;
    const uint32_t* prod_list;
    const double* prod_ve;
    const int32_t* prod_ev;
    uint32_t* bitmap[2];
    const uint32_t* prefix[2];
    pic_event* ev;
    int64_t ev_cap;
    const uint32_t* prod_c;   // weighted runs: ionized units per neutral slot
};

template <typename T>
__global__ void k_products(ProdArgs<T> a) {
    int64_t n = (int64_t)a.st->n_prod;
    if (n == 0) return;
    Species<T>& I = a.sp[PIC_ION];
    Species<T>& El = a.sp[PIC_ELECTRON];
    Species<T>& N = a.sp[PIC_NEUTRAL];
    int64_t base_i = (int64_t)a.st->n_slots[PIC_ION], base_e = (int64_t)a.st->n_slots[PIC_ELECTRON];
    bool room = base_i + n <= I.cap && base_e + n <= El.cap;
    uint32_t nid0 = (uint32_t)a.st->next_id;
    int64_t nimp = (int64_t)a.st->n_prod_kind[0];
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        uint32_t e = a.prod_list[p];
        int kind = e >> 31;
        uint32_t ib = e & 0x7FFFFFFFu;
        uint32_t id = N.id[ib];
        uint32_t w = a.bitmap[kind][id >> 5];
        int64_t r = (int64_t)a.prefix[kind][id >> 5] + __popc(w & ((1u << (id & 31)) - 1u));
        if (kind == 1) r += nimp;
        if (!room) continue;
        int64_t si = base_i + r, se = base_e + r;
        uint32_t id_ion = nid0 + 2u * (uint32_t)r, id_e = id_ion + 1u;
        T x = N.x[ib], y = N.y[ib], z = N.z[ib];
        I.x[si] = x;
        I.y[si] = y;
        I.z[si] = z;
        I.vx[si] = N.vx[ib];
        I.vy[si] = N.vy[ib];
        I.vz[si] = N.vz[ib];
        I.id[si] = id_ion;
        El.x[se] = x;
        El.y[se] = y;
        El.z[se] = z;
        El.vx[se] = (T)a.prod_ve[3 * (int64_t)ib + 0];
        El.vy[se] = (T)a.prod_ve[3 * (int64_t)ib + 1];
        El.vz[se] = (T)a.prod_ve[3 * (int64_t)ib + 2];
        El.id[se] = id_e;
        if (a.prod_c) {
            I.w[si] = a.prod_c[ib];
            El.w[se] = a.prod_c[ib];
        }
        int32_t q = a.prod_ev[ib];
        if (q >= 0 && q < a.ev_cap) {
            a.ev[q].new_ion = id_ion;
            a.ev[q].new_e = id_e;
        }
    }
}

// Second pass: clear the bitmap bits and free the neutral slots.
template <typename T>
__global__ void k_products_clear(ProdArgs<T> a) {
    int64_t n = (int64_t)a.st->n_prod;
    Species<T>& N = a.sp[PIC_NEUTRAL];
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        uint32_t e = a.prod_list[p];
        int kind = e >> 31;
        uint32_t ib = e & 0x7FFFFFFFu;
        uint32_t id = N.id[ib];
        atomicAnd(&a.bitmap[kind][id >> 5], ~(1u << (id & 31)));
        // the neutral loses the ionized units; without any left it is removed
        if (a.prod_c && N.w[ib] > a.prod_c[ib]) N.w[ib] -= a.prod_c[ib];
        else N.id[ib] = kDead;
    }
}

// ---------------------------------------------------------------------------
// Split-offs of partial collisions (Sec. 2.3.2): after the products, species
// by species in the order (species, parent id): the rank of a split-off among
// those of its species is read from the species' bitmap over parent ids and
// its word prefix counts; it takes the slot n_slots + rank and the id
// next_id + (split-offs of the species before) + rank, the parent's
// position, the collided units and their velocity; the parent keeps the rest.

template <typename T>
struct SplitArgs {
    Species<T> sp[3];
    DevState* st;
    uint32_t* list[3];
    const uint32_t* c[3];
    const double* v[3];
    uint32_t* bm[3];
    const uint32_t* pf[3];
};

template <typename T>
__global__ void k_splits(SplitArgs<T> a, int s) {
    const Species<T>& S = a.sp[s];
    const int64_t n = (int64_t)a.st->n_split[s];
    const int64_t base = (int64_t)a.st->n_slots[s];
    if (base + n > S.cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && n) atomicCAS(&a.st->error, 0, PIC_E_CAPACITY);
        return;
    }
    unsigned long long before = 0;
    for (int q = 0; q < s; ++q) before += a.st->n_split[q];
    const uint32_t id0 = (uint32_t)(a.st->next_id + before);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
        const uint32_t p = a.list[s][q];
        const uint32_t id = S.id[p];
        const uint32_t wd = a.bm[s][id >> 5];
        const int64_t r = (int64_t)a.pf[s][id >> 5] + __popc(wd & ((1u << (id & 31)) - 1u));
        if (r >= n) {  // a bit set that no split-off of the phase set
            atomicCAS(&a.st->error, 0, PIC_E_STATE);
            continue;
        }
        const int64_t m = base + r;
        const uint32_t c = a.c[s][p];
        S.x[m] = S.x[p];
        S.y[m] = S.y[p];
        S.z[m] = S.z[p];
        S.vx[m] = (T)a.v[s][3 * (int64_t)p + 0];
        S.vy[m] = (T)a.v[s][3 * (int64_t)p + 1];
        S.vz[m] = (T)a.v[s][3 * (int64_t)p + 2];
        S.id[m] = id0 + (uint32_t)r;
        S.w[m] = c;
        S.w[p] -= c;
    }
}

// clear the parents' bits once every rank is taken
template <typename T>
__global__ void k_splits_clear(SplitArgs<T> a, int s) {
    const Species<T>& S = a.sp[s];
    const int64_t n = (int64_t)a.st->n_split[s];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
        const uint32_t id = S.id[a.list[s][q]];
        atomicAnd(&a.bm[s][id >> 5], ~(1u << (id & 31)));
    }
}

__global__ void k_splits_finish(DevState* st, int64_t cap0, int64_t cap1, int64_t cap2) {
    const int64_t cap[3] = {cap0, cap1, cap2};
    unsigned long long tot = 0;
    for (int s = 0; s < 3; ++s) {
        if (st->n_slots[s] + st->n_split[s] > (unsigned long long)cap[s]) return;  // the error is set
        tot += st->n_split[s];
    }
    for (int s = 0; s < 3; ++s) st->n_slots[s] += st->n_split[s];
    st->next_id += tot;
    st->splits += tot;
}

__global__ void k_products_finish(DevState* st, int64_t cap_e, int64_t cap_i) {
    unsigned long long n = st->n_prod;
    if (st->n_slots[PIC_ION] + n > (unsigned long long)cap_i || st->n_slots[PIC_ELECTRON] + n > (unsigned long long)cap_e) {
        if (n) atomicCAS(&st->error, 0, PIC_E_CAPACITY);
        return;
    }
    st->n_slots[PIC_ION] += n;
    st->n_slots[PIC_ELECTRON] += n;
    st->next_id += 2ull * n;
}

// Number of bitmap words in use for the split-off ranks ((next_id + 31) / 32,
// 0 without split-offs).
__global__ void k_words_split(const DevState* st, uint32_t* words, int64_t maxw) {
    unsigned long long w = (st->next_id + 31ull) >> 5;
    if (st->n_split[0] + st->n_split[1] + st->n_split[2] == 0) w = 0;
    *words = (uint32_t)(w < (unsigned long long)maxw ? w : (unsigned long long)maxw);
}

// Number of bitmap words in use, (next_id + 31) / 32, for the device-sized scan.
__global__ void k_words(const DevState* st, uint32_t* words, int64_t maxw) {
    unsigned long long w = (st->next_id + 31ull) >> 5;
    if (st->n_prod == 0) w = 0;
    *words = (uint32_t)(w < (unsigned long long)maxw ? w : (unsigned long long)maxw);
}

// ---------------------------------------------------------------------------
// Reordering by cell: the alive particles of a species take the order of the
// (canonically sorted) cell bins; particles appended after the bins were
// built (products) follow in their order.

__global__ void k_sort_flags(int sp, const uint2* bins, const uint32_t* nbins, const uint32_t* const* ids,
                             uint32_t* flag, int64_t cap) {
    int64_t n = (int64_t)*nbins;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n && j < cap; j += stride) {
        uint32_t e = bins[j].x;
        uint32_t s = e >> 30;
        flag[j] = (s == (uint32_t)sp) && ids[s][e & 0x3FFFFFFFu] != kDead;
    }
}

template <typename T>
struct SortArgs {
    Species<T> s;
    int sp;
    const uint2* bins;
    const uint32_t* nbins;
    const uint32_t* flag;   // flags (before the scan)
    const uint32_t* rank;   // exclusive ranks
    const uint32_t* total;  // number of sorted particles
    T* tmp;                 // 6 * cap
    uint32_t* tmp_id;
    uint32_t* tmp_w;        // weighted runs
    DevState* st;
};

template <typename T>
__global__ void k_sort_gather(SortArgs<T> a) {
    int64_t n = (int64_t)*a.nbins;
    int64_t cap = a.s.cap;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        uint32_t e = a.bins[j].x;
        if ((e >> 30) != (uint32_t)a.sp) continue;
        uint32_t i = e & 0x3FFFFFFFu;
        if (a.s.id[i] == kDead) continue;
        int64_t d = a.rank[j];
        a.tmp[d] = a.s.x[i];
        a.tmp[cap + d] = a.s.y[i];
        a.tmp[2 * cap + d] = a.s.z[i];
        a.tmp[3 * cap + d] = a.s.vx[i];
        a.tmp[4 * cap + d] = a.s.vy[i];
        a.tmp[5 * cap + d] = a.s.vz[i];
        a.tmp_id[d] = a.s.id[i];
        if (a.s.w) a.tmp_w[d] = a.s.w[i];
    }
    // particles appended after the bins were built
    int64_t p0 = (int64_t)a.st->n_push[a.sp], p1 = (int64_t)a.st->n_slots[a.sp];
    int64_t ns = (int64_t)*a.total;
    for (int64_t i = p0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p1; i += stride) {
        int64_t d = ns + (i - p0);
        a.tmp[d] = a.s.x[i];
        a.tmp[cap + d] = a.s.y[i];
        a.tmp[2 * cap + d] = a.s.z[i];
        a.tmp[3 * cap + d] = a.s.vx[i];
        a.tmp[4 * cap + d] = a.s.vy[i];
        a.tmp[5 * cap + d] = a.s.vz[i];
        a.tmp_id[d] = a.s.id[i];
        if (a.s.w) a.tmp_w[d] = a.s.w[i];
    }
}

template <typename T>
__global__ void k_sort_copyback(SortArgs<T> a) {
    int64_t ns = (int64_t)*a.total + ((int64_t)a.st->n_slots[a.sp] - (int64_t)a.st->n_push[a.sp]);
    int64_t cap = a.s.cap;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += stride) {
        a.s.x[i] = a.tmp[i];
        a.s.y[i] = a.tmp[cap + i];
        a.s.z[i] = a.tmp[2 * cap + i];
        a.s.vx[i] = a.tmp[3 * cap + i];
        a.s.vy[i] = a.tmp[4 * cap + i];
        a.s.vz[i] = a.tmp[5 * cap + i];
        a.s.id[i] = a.tmp_id[i];
        if (a.s.w) a.s.w[i] = a.tmp_w[i];
    }
}

__global__ void k_sort_finish(DevState* st, int sp, const uint32_t* total) {
    unsigned long long ns = (unsigned long long)*total + (st->n_slots[sp] - st->n_push[sp]);
    st->n_slots[sp] = ns;
    st->n_push[sp] = 0;
}

// ---------------------------------------------------------------------------
// Per-step reset of the counters of one push/deposit pass.
__global__ void k_step_reset(DevState* st) {
    st->n_fi = 0;
    st->n_prod = 0;
    st->n_prod_kind[0] = st->n_prod_kind[1] = 0;
    st->n_ev = 0;
    st->n_big = 0;
    st->n_big2 = 0;
    for (int s = 0; s < 3; ++s) {
        st->smax_bits[s] = 0;
        st->n_push[s] = st->n_slots[s];
        st->n_split[s] = 0;
    }
}

// ---------------------------------------------------------------------------
// Host drivers

template <typename T>
static Species<T> species(pic_ctx* c, int s) {
    Species<T> r;
    r.x = (T*)c->buf.x[s];
    r.y = (T*)c->buf.y[s];
    r.z = (T*)c->buf.z[s];
    r.vx = (T*)c->buf.vx[s];
    r.vy = (T*)c->buf.vy[s];
    r.vz = (T*)c->buf.vz[s];
    r.id = c->buf.id[s];
    r.cap = c->buf.cap[s];
    r.w = c->cfg.weighted ? c->buf.w[s] : nullptr;
    return r;
}

static unsigned grid_for(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (unsigned)g;
}

// Grid of the push kernels (each block ends with a few device-wide atomics,
// so the block count stays bounded).
static unsigned grid_push(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (unsigned)g;
}

// Cell bins (counting sort of the keys), then the deposit.
template <typename T>
static hipError_t bin_t(pic_ctx* c) {
    const Grid& g = c->g;
    int tb = tic(c, PIC_T_BIN);
    hipError_t e = cell_bins(c);
    toc(c, tb);
    if (e != hipSuccess) return e;
    DepositArgs<T> d;
    d.e = species<T>(c, PIC_ELECTRON);
    d.ion = species<T>(c, PIC_ION);
    d.off = c->off;
    d.bins = c->bins;
    d.rho = c->buf.rho;
    d.g = g;
    d.st = c->st;
    int td = tic(c, PIC_T_DEPOSIT);
    hipLaunchKernelGGL(k_deposit_tiles<T>, dim3((unsigned)(g.nkeys / kTileCells)), dim3(kBlock), 0, c->stream, d);
    toc(c, td);
    c->bins_valid = 1;
    return hipGetLastError();
}

template <typename T>
static hipError_t particles_t(pic_ctx* c, bool move) {
    const pic_config& cf = c->cfg;
    hipLaunchKernelGGL(k_step_reset, dim3(1), dim3(1), 0, c->stream, c->st);
    (void)launch_zero(c->buf.rho, sizeof(int64_t) * c->g.nn, c->stream);
    for (int s = 0; s < 3; ++s) {
        PushArgs<T> a;
        a.s = species<T>(c, s);
        a.field = (const typename V4<T>::type*)c->buf.field;
        a.g = c->g;
        a.kq = (T)c->kq[s];
        a.rho = c->buf.rho;
        a.sign = s == PIC_ELECTRON ? -1 : 1;
        a.key = c->key[s];
        a.st = c->st;
        a.step = (uint32_t)c->step;
        a.seed = cf.seed;
        a.fi_list = c->fi_list;
        a.part = c->push_part;
        a.dpart = c->push_dpart;
        a.fi_cnt = c->fi_cnt;
        a.field0 = (move && c->circuit && s != PIC_NEUTRAL) ? (const typename V4<T>::type*)c->buf.field0 : nullptr;
        a.fi_thr = c->fi_thr;
        a.ebsi = c->ebsi;
        a.adk_c = c->adk_c;
        a.adk_e = 2.0 * c->adk_n - 1.0;
        a.x32 = pow(cf.xi, 1.5);
        a.dt_fs = cf.dt * 1e15;
        unsigned G = grid_push(a.s.cap);
        int t_all = s == 0 ? tic(c, PIC_T_PUSH) : -1;
        int t_e = s == 0 ? tic(c, PIC_T_PUSH_E) : -1;
        if (move) {
            if (s == 0) hipLaunchKernelGGL((k_push<T, 0, true>), dim3(G), dim3(kBlock), 0, c->stream, a);
            if (s == 1) hipLaunchKernelGGL((k_push<T, 1, true>), dim3(G), dim3(kBlock), 0, c->stream, a);
            if (s == 2) hipLaunchKernelGGL((k_push<T, 2, true>), dim3(G), dim3(kBlock), 0, c->stream, a);
        } else {
            if (s == 0) hipLaunchKernelGGL((k_push<T, 0, false>), dim3(G), dim3(kBlock), 0, c->stream, a);
            if (s == 1) hipLaunchKernelGGL((k_push<T, 1, false>), dim3(G), dim3(kBlock), 0, c->stream, a);
            if (s == 2) hipLaunchKernelGGL((k_push<T, 2, false>), dim3(G), dim3(kBlock), 0, c->stream, a);
        }
        toc(c, t_e);
        // the FP64 partials exist for moving ions (bombardment) and, with the
        // circuit, for moving charges (Shockley-Ramo current)
        const double sv = cf.h / cf.dt;
        const double* dp = (move && (s == PIC_ION || (s == PIC_ELECTRON && c->circuit))) ? c->push_dpart : nullptr;
        const double bsc = 0.5 * cf.m_ion * sv * sv;
        const double ssc = (s == PIC_ELECTRON ? -kQe : kQe) * sv;
        if (s == 0) hipLaunchKernelGGL(k_push_final<0>, dim3(1), dim3(kFinalBlock), 0, c->stream, c->st,
                                       (const uint32_t*)a.part, (int)G, dp, bsc, ssc);
        if (s == 1) hipLaunchKernelGGL(k_push_final<1>, dim3(1), dim3(kFinalBlock), 0, c->stream, c->st,
                                       (const uint32_t*)a.part, (int)G, dp, bsc, ssc);
        if (s == 2) hipLaunchKernelGGL(k_push_final<2>, dim3(1), dim3(kFinalBlock), 0, c->stream, c->st,
                                       (const uint32_t*)a.part, (int)G, (const double*)nullptr, bsc, ssc);
        if (s == 2) toc(c, c->push_all_handle);
        if (s == 0) c->push_all_handle = t_all;
    }
    if (move && c->circuit)
        hipLaunchKernelGGL(k_circuit, dim3(1), dim3(1), 0, c->stream, c->st, c->V0, cf.circuit_R, cf.circuit_C, cf.dt);
    return bin_t<T>(c);
}

hipError_t particles_phase(pic_ctx* c, bool move) {
    return c->cfg.precision == PIC_F32 ? particles_t<float>(c, move) : particles_t<double>(c, move);
}

// ---------------------------------------------------------------------------
// Same-species and Coulomb pairing (Table colls: Cu + Cu elastic, Coulomb
// collisions of the charged particles), on the bins of the push after the
// collisions and products of the step (unweighted runs). Per cell the
// particles of a species, in ascending id order, are rotated by
// floor(U_c N) (U_c from the cell, the step and the class) and paired
// consecutively. Cu + Cu: hard spheres, P = 1 - exp(-u n sigma_nn dt),
// n = N / h^3, isotropic scattering through Eq. du; neutrals with an event
// this step (or removed by it) keep their place but their pair is void, and
// with N odd the last one sits out. Coulomb (Takizuka-Abe): every pair turns
// its relative velocity by theta = 2 atan(delta), delta normal with variance
// e^4 n_L ln(Lambda) dt / (8 pi eps0^2 mu^2 u^3), through Eq. du; with N odd
// the first three collide pairwise with dt / 2 each; between electrons and
// ions each particle of the more numerous species meets one of the other,
// whose particles are reused cyclically (shifted by floor(U_c N_f)), with n_L
// the smaller density. Cells of up to kSmallCell particles take one thread;
// larger ones (listed by the collision scan) a wavefront, whose lanes take
// disjoint pairs.

template <typename T>
struct PairArgs {
    Species<T> sp[3];
    Grid g;
    const uint32_t* off;
    const uint2* bins;
    const uint32_t* big;     // cells of more than kSmallCell particles: up to kMidCell from the start
                             // (count st->n_big), more from the end (count st->n_big2)
    const uint32_t* nflag;   // neutral slot: step + 1 if it had an event this step
    DevState* st;
    uint32_t step;
    uint64_t seed;
    double h, dt, m_ion, sigma_nn, coulomb_log, sigma_rec;
    int nn, coul, rec;
    int64_t nc;
    // recombination: the charge is corrected here; the recombined ions are
    // listed (slot), flagged in a bitmap over ids, and their atoms' velocities
    // kept per ion slot until k_rec_place
    int64_t* rho;
    uint32_t* rec_list;
    double* rec_v;
    uint32_t* rec_bm;
    const uint32_t* rec_pf;
};

// Eq. du: Delta u = R^-1(theta, phi) [R^-1(theta', phi') - I] (0, 0, |u|)
__device__ inline void eq_du(const double u[3], double um, double ct2, double ph2, double du[3]) {
    const double up = sqrt(u[0] * u[0] + u[1] * u[1]);
    const double ct = u[2] / um, st = up / um;
    double cp = 1.0, sp = 0.0;
    if (up > 0.0) {
        cp = u[0] / up;
        sp = u[1] / up;
    }
    const double st2 = sqrt(1.0 - ct2 * ct2);
    double sp2, cp2;
    sincos(ph2, &sp2, &cp2);
    const double w0 = um * st2 * cp2, w1 = um * st2 * sp2, w2 = um * (ct2 - 1.0);
    du[0] = ct * cp * w0 - sp * w1 + st * cp * w2;
    du[1] = ct * sp * w0 + cp * w1 + st * sp * w2;
    du[2] = -st * w0 + ct * w2;
}

// One Takizuka-Abe scattering of (sa, ia) with (sb, ib) over dts at the
// density n_l, draws keyed by (subject, step, tag). Returns 1 if it turned.
template <typename T>
__device__ inline int ta_pair(const PairArgs<T>& a, uint32_t subject, uint32_t tag, int sa, uint32_t ia, int sb,
                              uint32_t ib, double n_l, double dts) {
    const Species<T>& A = a.sp[sa];
    const Species<T>& B = a.sp[sb];
    const double s = a.h / a.dt, g = a.dt / a.h;
    const double ma = sa == PIC_ELECTRON ? kMe : a.m_ion, mb = sb == PIC_ELECTRON ? kMe : a.m_ion;
    const double mu = ma * mb / (ma + mb);
    const double vA[3] = {(double)A.vx[ia], (double)A.vy[ia], (double)A.vz[ia]};
    const double vB[3] = {(double)B.vx[ib], (double)B.vy[ib], (double)B.vz[ib]};
    const double u[3] = {(vA[0] - vB[0]) * s, (vA[1] - vB[1]) * s, (vA[2] - vB[2]) * s};
    const double um = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    if (!(um > 0.0)) return 0;
    const double var =
        kQe * kQe * kQe * kQe * n_l * a.coulomb_log * dts / (8.0 * kPi * kEps0 * kEps0 * mu * mu * um * um * um);
    const Draw2 d0 = draw2(a.seed, subject, a.step, tag, 0);
    const Draw2 d1 = draw2(a.seed, subject, a.step, tag, 1);
    const double delta = sqrt(var) * sqrt(-2.0 * log(d0.a)) * cos(2.0 * kPi * d0.b);
    const double ct = (1.0 - delta * delta) / (1.0 + delta * delta);
    double du[3];
    eq_du(u, um, ct, 2.0 * kPi * d1.a, du);
    const double ka = mu / ma * g, kb = mu / mb * g;
    A.vx[ia] = (T)(vA[0] + ka * du[0]);
    A.vy[ia] = (T)(vA[1] + ka * du[1]);
    A.vz[ia] = (T)(vA[2] + ka * du[2]);
    B.vx[ib] = (T)(vB[0] - kb * du[0]);
    B.vy[ib] = (T)(vB[1] - kb * du[1]);
    B.vz[ib] = (T)(vB[2] - kb * du[2]);
    return 1;
}

// One Cu + Cu pair (slots ia, ib with ids ida, idb); returns 1 on a collision
template <typename T>
__device__ inline int nn_pair(const PairArgs<T>& a, uint32_t ia, uint32_t ida, uint32_t ib, uint32_t idb, double n) {
    const Species<T>& N = a.sp[PIC_NEUTRAL];
    if (N.id[ia] != ida || N.id[ib] != idb) return 0;                       // removed by an event
    if (a.nflag[ia] == a.step + 1u || a.nflag[ib] == a.step + 1u) return 0;  // had an event
    const double s = a.h / a.dt, g = a.dt / a.h;
    const double vA[3] = {(double)N.vx[ia], (double)N.vy[ia], (double)N.vz[ia]};
    const double vB[3] = {(double)N.vx[ib], (double)N.vy[ib], (double)N.vz[ib]};
    const double u[3] = {(vA[0] - vB[0]) * s, (vA[1] - vB[1]) * s, (vA[2] - vB[2]) * s};
    const double um = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const double P = -expm1(-um * n * a.sigma_nn * a.dt);
    if (!(draw2(a.seed, ida, a.step, kTagNN, 0).a < P)) return 0;
    const Draw2 r = draw2(a.seed, ida, a.step, kTagNN, 1);
    double du[3];
    eq_du(u, um, 2.0 * r.a - 1.0, 2.0 * kPi * r.b, du);
    const double k = 0.5 * g;  // mu / m = 1/2
    N.vx[ia] = (T)(vA[0] + k * du[0]);
    N.vy[ia] = (T)(vA[1] + k * du[1]);
    N.vz[ia] = (T)(vA[2] + k * du[2]);
    N.vx[ib] = (T)(vB[0] - k * du[0]);
    N.vy[ib] = (T)(vB[1] - k * du[1]);
    N.vz[ib] = (T)(vB[2] - k * du[2]);
    return 1;
}

__device__ inline int pair_shift(uint64_t seed, uint32_t lcell, uint32_t step, uint32_t tag, int N) {
    const Draw2 dc = draw2(seed, lcell, step, tag, 0);
    int sh = (int)floor(dc.a * (double)N);
    return sh > N - 1 ? N - 1 : sh;
}

// The classes of one cell whose entries (species << 30 | slot, ids) are
// sorted by (species, id): kv[t] = species << 32 | id, ev[t] = the value.
// lane / lanes split the disjoint pairs (1 / 1 for one thread per cell);
// sync() orders the rounds that reuse a particle.
// One electron-ion pair of the recombination class; returns 1 if it
// recombined (the electron is removed at once, the ion by k_rec_clear)
template <typename T>
__device__ inline int rec_pair(const PairArgs<T>& a, uint32_t pid, uint32_t ie, uint32_t ii, double n) {
    const Species<T>& E = a.sp[PIC_ELECTRON];
    const Species<T>& I = a.sp[PIC_ION];
    const double s = a.h / a.dt;
    const double vE[3] = {(double)E.vx[ie], (double)E.vy[ie], (double)E.vz[ie]};
    const double vI[3] = {(double)I.vx[ii], (double)I.vy[ii], (double)I.vz[ii]};
    const double u[3] = {(vE[0] - vI[0]) * s, (vE[1] - vI[1]) * s, (vE[2] - vI[2]) * s};
    const double um = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const double P = -expm1(-um * n * a.sigma_rec * a.dt);
    if (!(draw2(a.seed, pid, a.step, kTagRec, 0).a < P)) return 0;
    const double mt = kMe + a.m_ion;
    for (int k = 0; k < 3; ++k) a.rec_v[3 * (int64_t)ii + k] = (kMe * vE[k] + a.m_ion * vI[k]) / mt;
    const uint32_t idi = I.id[ii];
    atomicOr(&a.rec_bm[idi >> 5], 1u << (idi & 31));
    const unsigned long long q = atomicAdd(&a.st->n_rec, 1ull);
    a.rec_list[q] = ii;
    // the deposit of this step counted both charges
    unsigned long long* rho = (unsigned long long*)a.rho;
    deposit_one(a.g, rho, (double)E.x[ie], (double)E.y[ie], (double)E.z[ie], 1);
    deposit_one(a.g, rho, (double)I.x[ii], (double)I.y[ii], (double)I.z[ii], -1);
    E.id[ie] = kDead;
    return 1;
}

template <typename T, typename SL, typename ID, typename Sync>
__device__ inline void pair_coulomb(const PairArgs<T>& a, const int b0[4], uint32_t lc, double vol, const SL& slot,
                                    const ID& idof, int lane, int lanes, Sync sync, int cnt[3]) {
    for (int sp = PIC_ELECTRON; sp <= PIC_ION; ++sp) {
        const int o = b0[sp], N = b0[sp + 1] - o;
        if (N < 2) continue;
        const int sh = pair_shift(a.seed, lc, a.step, sp == PIC_ELECTRON ? kTagPairEE : kTagPairII, N);
        const double n = (double)N / vol;
        const auto q = [&](int j) { return o + (sh + j) % N; };
        int j0 = 0;
        if (N % 2 == 1) {
            if (lane == 0) {
                cnt[1] += ta_pair(a, idof(q(0)), kTagCoul, sp, slot(q(0)), sp, slot(q(1)), n, 0.5 * a.dt);
                cnt[1] += ta_pair(a, idof(q(1)), kTagCoul, sp, slot(q(1)), sp, slot(q(2)), n, 0.5 * a.dt);
                cnt[1] += ta_pair(a, idof(q(2)), kTagCoul, sp, slot(q(2)), sp, slot(q(0)), n, 0.5 * a.dt);
            }
            sync();
            j0 = 3;
        }
        for (int j = j0 + 2 * lane; j + 1 < N; j += 2 * lanes)
            cnt[1] += ta_pair(a, idof(q(j)), kTagCoul, sp, slot(q(j)), sp, slot(q(j + 1)), n, a.dt);
        sync();
    }
    const int oe = b0[PIC_ELECTRON], NE = b0[PIC_ELECTRON + 1] - oe;
    const int oi = b0[PIC_ION], NI = b0[PIC_ION + 1] - oi;
    if (NE > 0 && NI > 0) {
        const bool e_more = NE >= NI;
        const int oM = e_more ? oe : oi, NM = e_more ? NE : NI, oF = e_more ? oi : oe, NF = e_more ? NI : NE;
        const int sh = pair_shift(a.seed, lc, a.step, kTagPairEI, NF);
        const double n_l = (double)NF / vol;
        // rounds of NF pairs: within a round every particle of the fewer
        // species appears once
        for (int r0 = 0; r0 < NM; r0 += NF) {
            const int r1 = r0 + NF < NM ? r0 + NF : NM;
            for (int i = r0 + lane; i < r1; i += lanes) {
                const int tm = oM + i, tf = oF + (sh + i) % NF;
                const int te = e_more ? tm : tf, ti = e_more ? tf : tm;
                cnt[1] += ta_pair(a, idof(tm), kTagCoulEI, PIC_ELECTRON, slot(te), PIC_ION, slot(ti), n_l, a.dt);
            }
            sync();
        }
    }
}

template <typename T, typename KV, typename EV, typename Sync>
__device__ inline void pair_classes(const PairArgs<T>& a, uint32_t cell, const KV& kv, const EV& ev, int n, int lane,
                                    int lanes, Sync sync, int cnt[3]) {
    int b0[4] = {0, 0, 0, 0};
    for (int t = 0; t < n; ++t) b0[(int)(kv(t) >> 32) + 1] = t + 1;
    for (int s = 1; s < 4; ++s) b0[s] = b0[s] > b0[s - 1] ? b0[s] : b0[s - 1];
    const uint32_t lc = linear_cell(a.g, cell);
    const double vol = a.h * a.h * a.h;
    const auto slot = [&](int t) { return ev(t) & 0x3FFFFFFFu; };
    const auto idof = [&](int t) { return (uint32_t)(kv(t) & 0xFFFFFFFFu); };
    if (a.nn) {
        const int o = b0[PIC_NEUTRAL], N = b0[PIC_NEUTRAL + 1] - o;
        if (N >= 2) {
            const int sh = pair_shift(a.seed, lc, a.step, kTagPairNN, N);
            const double n = (double)N / vol;
            for (int j = 2 * lane; j + 1 < N; j += 2 * lanes) {
                const int ta = o + (sh + j) % N, tb = o + (sh + j + 1) % N;
                cnt[0] += nn_pair(a, slot(ta), idof(ta), slot(tb), idof(tb), n);
            }
            sync();
        }
    }
    if (a.coul) pair_coulomb(a, b0, lc, vol, slot, idof, lane, lanes, sync, cnt);
    if (a.rec) {
        const int oe = b0[PIC_ELECTRON], NE = b0[PIC_ELECTRON + 1] - oe;
        const int oi = b0[PIC_ION], NI = b0[PIC_ION + 1] - oi;
        if (NE > 0 && NI > 0) {
            const bool ion_proj = NI <= NE;
            const int oP = ion_proj ? oi : oe, NP = ion_proj ? NI : NE, oT = ion_proj ? oe : oi, NT = ion_proj ? NE : NI;
            const int sh = pair_shift(a.seed, lc, a.step, kTagPairRec, NT);
            const double n = (double)NT / vol;
            for (int i = lane; i < NP; i += lanes) {
                const int tp = oP + i, tt = oT + (sh + i) % NT;
                cnt[2] += rec_pair(a, idof(tp), slot(ion_proj ? tt : tp), slot(ion_proj ? tp : tt), n);
            }
            sync();
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_pair_small(PairArgs<T> a) {
    int cnt[3] = {0, 0, 0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < a.nc; c += stride) {
        const uint32_t o0 = a.off[c];
        const int n = (int)(a.off[c + 1] - o0);
        if (n < 2 || n > kSmallCell) continue;
        uint64_t kk[kSmallCell];
        uint32_t ee[kSmallCell];
        for (int t = 0; t < n; ++t) {
            const uint2 be = a.bins[o0 + t];
            const uint64_t k = ((uint64_t)(be.x >> 30) << 32) | be.y;
            int u = t;
            while (u > 0 && kk[u - 1] > k) {
                kk[u] = kk[u - 1];
                ee[u] = ee[u - 1];
                --u;
            }
            kk[u] = k;
            ee[u] = be.x;
        }
        pair_classes(
            a, (uint32_t)c, [&](int t) { return kk[t]; }, [&](int t) { return ee[t]; }, n, 0, 1, [] {}, cnt);
    }
    __shared__ int sh[kBlock / 64];
    const int t0 = block_sum(cnt[0], sh);
    const int t1 = block_sum(cnt[1], sh);
    if (threadIdx.x == 0) {
        if (t0) atomicAdd(&a.st->nn_events, (unsigned long long)t0);
        if (t1) atomicAdd(&a.st->coulomb_pairs, (unsigned long long)t1);
    }
}

// one wavefront (block of 64) per listed big cell: CAP = kMidCell for the
// cells listed from the start of the list, CAP = kBigCell for those from its
// end
template <typename T, int CAP>
__global__ __launch_bounds__(64) void k_pair_big(PairArgs<T> a) {
    __shared__ uint64_t kk[CAP];
    __shared__ uint32_t ee[CAP];
    constexpr bool kBack = CAP > kMidCell;
    const int lane = threadIdx.x;
    int cnt[3] = {0, 0, 0};
    const int64_t nbig = (int64_t)(kBack ? a.st->n_big2 : a.st->n_big);
    for (int64_t b = blockIdx.x; b < nbig; b += gridDim.x) {
        const uint32_t c = kBack ? a.big[a.nc - 1 - b] : a.big[b];
        const uint32_t o0 = a.off[c];
        const int n = (int)(a.off[c + 1] - o0);
        if (n > kBigCell) {  // not supported by the pairing of this kernel
            if (lane == 0) atomicCAS(&a.st->error, 0, PIC_E_CAPACITY);
            continue;
        }
        int P = 1;
        while (P < n) P <<= 1;
        for (int t = lane; t < P; t += 64) {
            if (t < n) {
                const uint2 be = a.bins[o0 + t];
                kk[t] = ((uint64_t)(be.x >> 30) << 32) | be.y;
                ee[t] = be.x;
            } else {
                kk[t] = ~0ull;
                ee[t] = 0;
            }
        }
        __syncthreads();
        for (int k = 2; k <= P; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int t = lane; t < P; t += 64) {
                    const int u = t ^ j;
                    if (u > t) {
                        const bool up = (t & k) == 0;
                        const uint64_t x = kk[t], y = kk[u];
                        if ((x > y) == up) {
                            kk[t] = y;
                            kk[u] = x;
                            const uint32_t ex = ee[t];
                            ee[t] = ee[u];
                            ee[u] = ex;
                        }
                    }
                }
                __syncthreads();
            }
        }
        pair_classes(
            a, c, [&](int t) { return kk[t]; }, [&](int t) { return ee[t]; }, n, lane, 64,
            [] { __syncthreads(); }, cnt);
        __syncthreads();
    }
    const int t0 = wave_sum(cnt[0]), t1 = wave_sum(cnt[1]);
    if (lane == 0) {
        if (t0) atomicAdd(&a.st->nn_events, (unsigned long long)t0);
        if (t1) atomicAdd(&a.st->coulomb_pairs, (unsigned long long)t1);
    }
}

// The atoms of the recombinations of the phase, in ascending order of the
// recombined ions' ids (their ranks in the bitmap), after the other
// products; then the ions are removed and the bits cleared.
template <typename T>
__global__ void k_rec_place(PairArgs<T> a) {
    const Species<T>& I = a.sp[PIC_ION];
    const Species<T>& N = a.sp[PIC_NEUTRAL];
    const int64_t n = (int64_t)a.st->n_rec;
    const int64_t base = (int64_t)a.st->n_slots[PIC_NEUTRAL];
    if (base + n > N.cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && n) atomicCAS(&a.st->error, 0, PIC_E_CAPACITY);
        return;
    }
    const uint32_t id0 = (uint32_t)a.st->next_id;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
        const uint32_t p = a.rec_list[q];
        const uint32_t id = I.id[p];
        const uint32_t wd = a.rec_bm[id >> 5];
        const int64_t r = (int64_t)a.rec_pf[id >> 5] + __popc(wd & ((1u << (id & 31)) - 1u));
        if (r >= n) {  // a bit set that no recombination of the phase set
            atomicCAS(&a.st->error, 0, PIC_E_STATE);
            continue;
        }
        const int64_t m = base + r;
        N.x[m] = I.x[p];
        N.y[m] = I.y[p];
        N.z[m] = I.z[p];
        N.vx[m] = (T)a.rec_v[3 * (int64_t)p + 0];
        N.vy[m] = (T)a.rec_v[3 * (int64_t)p + 1];
        N.vz[m] = (T)a.rec_v[3 * (int64_t)p + 2];
        N.id[m] = id0 + (uint32_t)r;
        if (N.w) N.w[m] = 1u;
    }
}

template <typename T>
__global__ void k_rec_clear(PairArgs<T> a) {
    const Species<T>& I = a.sp[PIC_ION];
    const int64_t n = (int64_t)a.st->n_rec;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
        const uint32_t p = a.rec_list[q];
        const uint32_t id = I.id[p];
        atomicAnd(&a.rec_bm[id >> 5], ~(1u << (id & 31)));
        I.id[p] = kDead;
    }
}

__global__ void k_rec_finish(DevState* st, int64_t cap_n) {
    const unsigned long long n = st->n_rec;
    st->n_rec = 0;
    if (st->n_slots[PIC_NEUTRAL] + n > (unsigned long long)cap_n) return;  // the error is set
    st->n_slots[PIC_NEUTRAL] += n;
    st->next_id += n;
    st->recombinations += n;
}

__global__ void k_words_rec(const DevState* st, uint32_t* words, int64_t maxw) {
    unsigned long long w = (st->next_id + 31ull) >> 5;
    if (st->n_rec == 0) w = 0;
    *words = (uint32_t)(w < (unsigned long long)maxw ? w : (unsigned long long)maxw);
}

// ---------------------------------------------------------------------------
// Merging of superparticles (Sec. 2.3.2, the centre-of-mass merge of two
// superparticles of one type). The paper does not say which pairs merge:
// per cell and species, the superparticles binned by this step's push that
// are still alive are ranked by id; with N > merge_max of them, ranks (0,1),
// (2,3), ... up to k = min(floor(N/2), N - merge_max) pairs merge, keeping
// the lower id, unless the summed weight would exceed w_max. One kernel picks
// the partner of every rank-even entry (reading only), a second applies the
// merges, so the picks never see a half-merged cell. The node charge was
// deposited before the collisions; the merge subtracts the two deposits and
// adds the merged one, integer sums, so the result equals a fresh deposit.

template <typename T>
struct MergeArgs {
    Species<T> sp[3];
    Grid g;
    const uint32_t* off;    // cell offsets of the push's binning
    const uint2* bins;      // {species << 30 | slot, id} in cell order
    const uint32_t* key[3]; // cell key of every slot from the push
    uint32_t* pick;         // per bin entry: the partner's entry, or kDead
    int64_t* rho;
    DevState* st;
    int64_t entries_cap;
    uint32_t merge_max, w_max;
};

template <typename T>
__device__ inline bool merge_alive(const MergeArgs<T>& a, uint2 e, uint32_t s) {
    return (e.x >> 30) == s && a.sp[s].id[e.x & 0x3FFFFFFFu] == e.y;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_merge_pick(MergeArgs<T> a) {
    const int64_t total = a.off[a.g.nkeys];
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < a.entries_cap;
         b += (int64_t)gridDim.x * blockDim.x) {
        if (b >= total) break;
        const uint2 e = a.bins[b];
        const uint32_t s = e.x >> 30;
        uint32_t partner = kDead;
        if (merge_alive(a, e, s)) {
            const uint32_t k = a.key[s][e.x & 0x3FFFFFFFu];
            const uint32_t o0 = a.off[k], o1 = a.off[k + 1];
            uint32_t n = 0, r = 0, next_id = kDead, next_entry = kDead;
            for (uint32_t j = o0; j < o1; ++j) {
                const uint2 f = a.bins[j];
                if (!merge_alive(a, f, s)) continue;
                ++n;
                if (f.y < e.y) ++r;
                if (f.y > e.y && f.y < next_id) {
                    next_id = f.y;
                    next_entry = j;
                }
            }
            if (n > a.merge_max && (r & 1u) == 0u) {
                const uint32_t pairs = min(n / 2, n - a.merge_max);
                if (r / 2 < pairs) partner = next_entry;
            }
        }
        a.pick[b] = partner;
    }
}

// adds sg charges at (X, Y, Z) with the quantized CIC weights of the deposit
__device__ inline void deposit_one(const Grid& g, unsigned long long* rho, double X, double Y, double Z,
                                   int64_t sg) {
    const int ci = clampi((int)floor(X), 0, g.nx - 2), cj = clampi((int)floor(Y), 0, g.ny - 2),
              ck = clampi((int)floor(Z), 0, g.nz - 2);
    const int64_t qx = quantize(X - ci, 13), qy = quantize(Y - cj, 13), qz = quantize(Z - ck, 14);
    const int64_t w[2][3] = {{8192 - qx, 8192 - qy, 16384 - qz}, {qx, qy, qz}};
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int dx = t & 1, dy = (t >> 1) & 1, dz = (t >> 2) & 1;
        const int64_t v = sg * w[dx][0] * w[dy][1] * w[dz][2];
        atomicAdd(rho + ((int64_t)(ck + dz) * g.ny + cj + dy) * g.nx + ci + dx, (unsigned long long)v);
    }
}

// (wa a + wb b) / (wa + wb), evaluated as written (no contraction)
__device__ inline double merge_mean(double wa, double va, double wb, double vb) {
#pragma clang fp contract(off)
    return (wa * va + wb * vb) / (wa + wb);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_merge_apply(MergeArgs<T> a) {
    const int64_t total = a.off[a.g.nkeys];
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < a.entries_cap;
         b += (int64_t)gridDim.x * blockDim.x) {
        if (b >= total) break;
        const uint32_t j = a.pick[b];
        if (j == kDead) continue;
        const uint2 e = a.bins[b];
        const uint32_t s = e.x >> 30;
        const uint32_t i = e.x & 0x3FFFFFFFu, p = a.bins[j].x & 0x3FFFFFFFu;
        const Species<T>& P = a.sp[s];
        const uint32_t wa = P.w[i], wb = P.w[p];
        if ((uint64_t)wa + wb > (uint64_t)a.w_max) continue;
        const double fa = (double)wa, fb = (double)wb;
        const double xa = (double)P.x[i], ya = (double)P.y[i], za = (double)P.z[i];
        const double xb = (double)P.x[p], yb = (double)P.y[p], zb = (double)P.z[p];
        const T xm = (T)merge_mean(fa, xa, fb, xb), ym = (T)merge_mean(fa, ya, fb, yb),
                zm = (T)merge_mean(fa, za, fb, zb);
        P.vx[i] = (T)merge_mean(fa, (double)P.vx[i], fb, (double)P.vx[p]);
        P.vy[i] = (T)merge_mean(fa, (double)P.vy[i], fb, (double)P.vy[p]);
        P.vz[i] = (T)merge_mean(fa, (double)P.vz[i], fb, (double)P.vz[p]);
        P.x[i] = xm;
        P.y[i] = ym;
        P.z[i] = zm;
        P.w[i] = wa + wb;
        P.id[p] = kDead;
        atomicAdd(&a.st->merges[s], 1ull);
        if (s != PIC_NEUTRAL) {
            const int64_t sg = s == PIC_ELECTRON ? -1 : 1;
            unsigned long long* rho = (unsigned long long*)a.rho;
            deposit_one(a.g, rho, xa, ya, za, -sg * (int64_t)wa);
            deposit_one(a.g, rho, xb, yb, zb, -sg * (int64_t)wb);
            deposit_one(a.g, rho, (double)xm, (double)ym, (double)zm, sg * ((int64_t)wa + wb));
        }
    }
}

template <typename T>
static hipError_t collide_t(pic_ctx* c, bool record) {
    const pic_config& cf = c->cfg;
    const Grid& g = c->g;
    hipError_t e;
    bool resort = cf.sort_every > 0 && (c->need_sort || ((c->collide_count + 1) % cf.sort_every) == 0);
    c->need_sort = 0;
    MccArgs<T> a;
    for (int s = 0; s < 3; ++s) a.sp[s] = species<T>(c, s);
    a.g = g;
    a.off = c->off;
    a.bins = c->bins;
    a.nc = g.nkeys;
    a.big = c->big;
    a.mcc_list = c->mcc_list;
    a.mcc_count = c->mcc_count;
    a.mcc_dense = c->mcc_dense;
    a.mcc_total = c->dyn + 8;
    a.st = c->st;
    a.step = (uint32_t)c->step;
    a.seed = cf.seed;
    a.h = cf.h;
    a.dt = cf.dt;
    a.m_ion = cf.m_ion;
    a.xi = cf.xi;
    a.xs = c->xs;
    a.xs_n = cf.xs_n;
    a.xs_emin = cf.xs_emin;
    a.xs_lnr = log(cf.xs_emax / cf.xs_emin);
    a.nflag = c->nflag;
    a.bitmap_imp = c->bitmap[0];
    a.prod_list = c->prod_list;
    a.prod_ve = c->prod_ve;
    a.prod_ev = c->prod_ev;
    a.ev = c->ev;
    a.ev_cap = c->ev_cap;
    a.record = record ? 1 : 0;
    a.write_sorted = resort ? 1 : 0;
    a.weighted = cf.weighted ? 1 : 0;
    a.prod_c = c->prod_c;
    a.fi_cnt = c->fi_cnt;
    for (int s = 0; s < 3; ++s) {
        a.split_list[s] = c->split_list[s];
        a.split_c[s] = c->split_c[s];
        a.split_v[s] = c->split_v[s];
        a.split_bm[s] = c->split_bm[s];
    }
    int tm = tic(c, PIC_T_MCC);
    // the scan and the compaction take the same grid (a wavefront of the
    // second copies the segment of the same wavefront of the first)
    // on the side stream (concurrent with the Poisson solve) the collision
    // kernels take a part of the GPU only, so the solve keeps most of it
    const bool side = c->stream == c->side_stream;
    const unsigned gm = side ? std::min(grid_for(g.nkeys), 1024u) : grid_for(g.nkeys);
    hipLaunchKernelGGL(k_mcc_small<T>, dim3(gm), dim3(kBlock), 0, c->stream, a);
    e = scan_u32(c, c->mcc_count, c->mcc_count, (int64_t)gm * (kBlock / 64), nullptr, c->dyn + 8, false, false);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mcc_compact<T>, dim3(gm), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL(k_mcc_cells<T>, dim3(side ? 256 : 2048), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL((k_mcc_big<T, kMidCell>), dim3(8192), dim3(64), 0, c->stream, a);
    hipLaunchKernelGGL((k_mcc_big<T, kBigCell>), dim3(1024), dim3(64), 0, c->stream, a);
    hipLaunchKernelGGL(k_mcc_huge<T>, dim3(64), dim3(kHugeThreads), 0, c->stream, a, c->rank_flag);
    toc(c, tm);
    hipLaunchKernelGGL(k_fi_resolve<T>, dim3(grid_for(c->buf.cap[2])), dim3(kBlock), 0, c->stream, a, c->fi_list,
                       c->bitmap[1]);
    // products
    uint32_t* words = c->dyn;
    hipLaunchKernelGGL(k_words, dim3(1), dim3(1), 0, c->stream, c->st, words, c->bm_words);
    for (int k = 0; k < 2; ++k) {
        e = scan_u32(c, c->bitmap[k], c->bm_prefix[k], c->bm_words, words, nullptr, false, true);
        if (e != hipSuccess) return e;
    }
    ProdArgs<T> p;
    for (int s = 0; s < 3; ++s) p.sp[s] = species<T>(c, s);
    p.st = c->st;
    p.prod_list = c->prod_list;
    p.prod_ve = c->prod_ve;
    p.prod_ev = c->prod_ev;
    p.bitmap[0] = c->bitmap[0];
    p.bitmap[1] = c->bitmap[1];
    p.prefix[0] = c->bm_prefix[0];
    p.prefix[1] = c->bm_prefix[1];
    p.ev = c->ev;
    p.ev_cap = c->ev_cap;
    p.prod_c = cf.weighted ? c->prod_c : nullptr;
    unsigned Gp = grid_for(c->buf.cap[2]);
    hipLaunchKernelGGL(k_products<T>, dim3(Gp), dim3(kBlock), 0, c->stream, p);
    hipLaunchKernelGGL(k_products_clear<T>, dim3(Gp), dim3(kBlock), 0, c->stream, p);
    hipLaunchKernelGGL(k_products_finish, dim3(1), dim3(1), 0, c->stream, c->st, c->buf.cap[0], c->buf.cap[1]);
    if (cf.weighted) {
        // split-offs of partial collisions, after the products
        uint32_t* wsplit = c->dyn + 2;
        hipLaunchKernelGGL(k_words_split, dim3(1), dim3(1), 0, c->stream, c->st, wsplit, c->bm_words);
        SplitArgs<T> sa;
        for (int s = 0; s < 3; ++s) {
            e = scan_u32(c, c->split_bm[s], c->split_pf[s], c->bm_words, wsplit, nullptr, false, true);
            if (e != hipSuccess) return e;
            sa.sp[s] = species<T>(c, s);
            sa.list[s] = c->split_list[s];
            sa.c[s] = c->split_c[s];
            sa.v[s] = c->split_v[s];
            sa.bm[s] = c->split_bm[s];
            sa.pf[s] = c->split_pf[s];
        }
        sa.st = c->st;
        for (int s = 0; s < 3; ++s)
            hipLaunchKernelGGL(k_splits<T>, dim3(grid_for(c->buf.cap[s])), dim3(kBlock), 0, c->stream, sa, s);
        for (int s = 0; s < 3; ++s)
            hipLaunchKernelGGL(k_splits_clear<T>, dim3(grid_for(c->buf.cap[s])), dim3(kBlock), 0, c->stream, sa, s);
        hipLaunchKernelGGL(k_splits_finish, dim3(1), dim3(1), 0, c->stream, c->st, c->buf.cap[0], c->buf.cap[1],
                           c->buf.cap[2]);
    }
    if (cf.same_species) {
        PairArgs<T> pa;
        for (int s = 0; s < 3; ++s) pa.sp[s] = species<T>(c, s);
        pa.g = g;
        pa.off = c->off;
        pa.bins = c->bins;
        pa.big = c->big;
        pa.nflag = c->nflag;
        pa.st = c->st;
        pa.step = (uint32_t)c->step;
        pa.seed = cf.seed;
        pa.h = cf.h;
        pa.dt = cf.dt;
        pa.m_ion = cf.m_ion;
        pa.sigma_nn = cf.sigma_nn;
        pa.coulomb_log = cf.coulomb_log;
        pa.sigma_rec = cf.sigma_rec;
        pa.nn = (cf.same_species & 1) ? 1 : 0;
        pa.coul = (cf.same_species & 2) ? 1 : 0;
        pa.rec = (cf.same_species & 4) ? 1 : 0;
        pa.nc = g.nkeys;
        pa.rho = c->buf.rho;
        pa.rec_list = c->rec_list;
        pa.rec_v = c->rec_v;
        pa.rec_bm = c->rec_bm;
        pa.rec_pf = c->rec_pf;
        hipLaunchKernelGGL(k_pair_small<T>, dim3(side ? std::min(grid_for(g.nkeys), 1024u) : grid_for(g.nkeys)),
                           dim3(kBlock), 0, c->stream, pa);
        hipLaunchKernelGGL((k_pair_big<T, kMidCell>), dim3(8192), dim3(64), 0, c->stream, pa);
        hipLaunchKernelGGL((k_pair_big<T, kBigCell>), dim3(256), dim3(64), 0, c->stream, pa);
        if (pa.rec) {
            uint32_t* wrec = c->dyn + 16;
            hipLaunchKernelGGL(k_words_rec, dim3(1), dim3(1), 0, c->stream, c->st, wrec, c->bm_words);
            e = scan_u32(c, c->rec_bm, c->rec_pf, c->bm_words, wrec, nullptr, false, true);
            if (e != hipSuccess) return e;
            const unsigned Gr = grid_for(c->buf.cap[1]);
            hipLaunchKernelGGL(k_rec_place<T>, dim3(Gr), dim3(kBlock), 0, c->stream, pa);
            hipLaunchKernelGGL(k_rec_clear<T>, dim3(Gr), dim3(kBlock), 0, c->stream, pa);
            hipLaunchKernelGGL(k_rec_finish, dim3(1), dim3(1), 0, c->stream, c->st, c->buf.cap[2]);
        }
    }
    if (merge_step(c)) {
        MergeArgs<T> ma;
        for (int s = 0; s < 3; ++s) ma.sp[s] = species<T>(c, s);
        ma.g = g;
        ma.off = c->off;
        ma.bins = c->bins;
        for (int s = 0; s < 3; ++s) ma.key[s] = c->key[s];
        ma.pick = c->rank_flag;
        ma.rho = c->buf.rho;
        ma.st = c->st;
        ma.entries_cap = c->buf.cap[0] + c->buf.cap[1] + c->buf.cap[2];
        ma.merge_max = (uint32_t)cf.merge_max;
        ma.w_max = (uint32_t)(cf.w_max > 1 ? cf.w_max : 1);
        const unsigned G = grid_for(ma.entries_cap);
        hipLaunchKernelGGL(k_merge_pick<T>, dim3(G), dim3(kBlock), 0, c->stream, ma);
        hipLaunchKernelGGL(k_merge_apply<T>, dim3(G), dim3(kBlock), 0, c->stream, ma);
    }
    if (resort) {
        uint32_t* flag = c->rank_flag;
        int64_t capsum = c->buf.cap[0] + c->buf.cap[1] + c->buf.cap[2];
        for (int s = 0; s < 3; ++s) {
            hipLaunchKernelGGL(k_sort_flags, dim3(grid_for(capsum)), dim3(kBlock), 0, c->stream, s, c->bins,
                               c->off + g.nkeys, (const uint32_t* const*)c->id_ptrs, flag, capsum);
            e = scan_u32(c, flag, c->rank, capsum, c->off + g.nkeys, c->dyn + 1, false, false);
            if (e != hipSuccess) return e;
            SortArgs<T> sa;
            sa.s = species<T>(c, s);
            sa.sp = s;
            sa.bins = c->bins;
            sa.nbins = c->off + g.nkeys;
            sa.flag = flag;
            sa.rank = c->rank;
            sa.total = c->dyn + 1;
            sa.tmp = (T*)c->tmp;
            sa.tmp_id = (uint32_t*)((T*)c->tmp + 6 * c->tmp_cap);
            sa.tmp_w = sa.tmp_id + c->tmp_cap;
            sa.st = c->st;
            hipLaunchKernelGGL(k_sort_gather<T>, dim3(grid_for(capsum)), dim3(kBlock), 0, c->stream, sa);
            hipLaunchKernelGGL(k_sort_copyback<T>, dim3(grid_for(sa.s.cap)), dim3(kBlock), 0, c->stream, sa);
            hipLaunchKernelGGL(k_sort_finish, dim3(1), dim3(1), 0, c->stream, c->st, s, c->dyn + 1);
        }
    }
    c->collide_count++;
    c->bins_valid = 0;
    return hipGetLastError();
}

hipError_t collide_phase(pic_ctx* c, bool record) {
    return c->cfg.precision == PIC_F32 ? collide_t<float>(c, record) : collide_t<double>(c, record);
}

// ---------------------------------------------------------------------------
// Surface injection (Sec. 2.3.1), per patch of the analytic tip surface;
// floor(N) particles plus one with probability frac(N) are placed uniformly
// on the patch, 10^-3 spacings outside the surface; ids follow patch order.
//  - Field emission (kind 0): the field one spacing out along the normal
//    gives the Murphy-Good current density J, N = J A dt / e electrons, at
//    rest.
//  - Evaporation (kind 1): the Clausius-Clapeyron flux at the prescribed
//    surface temperature (taken on the host) gives N = flux A dt neutrals,
//    leaving with a Rayleigh-distributed normal speed and Gaussian tangential
//    components (the Maxwellian of the surface temperature, flux weighted).

struct InjArgs {
    Grid g;
    const double* phi;
    int rings, naz;
    int64_t npatch;
    double fn_a, fn_b, fn_cs2, phi_w, h, dt;
    uint64_t seed;
    uint32_t step;
    DevState* st;
    int64_t cap;
    double phi_w15;    // phi_w^1.5, taken on the host
    uint32_t* cnt;     // count of each patch
    double* part;      // per count block: expected count, clamped patches
    int kind;          // 0 field emission (electrons), 1 evaporation (neutrals)
    double evap_flux;  // evaporation flux [1/(m^2 s)]
    double vsig;       // evaporation: sqrt(k_B T / m) in grid units per step
    // superparticle weights of evaporated neutrals (Sec. 2.3.2), weighted runs
    int weighted, w_max;
    double n_max;
    const uint32_t* off;  // cell offsets of the last binning (tile-major keys)
    uint2* wk;            // per patch: {weight, atoms}
};

// Weight of the superparticles injected at a surface location (Sec. 2.3.2):
// min(ceil(max(1, sqrt((n_cell / n_max) N_inj))), w_max), w_min = 1, n_cell the
// superparticle density of the cell of the field point at the last binning.
__device__ inline uint32_t inject_weight(const InjArgs& a, int64_t atoms, uint32_t cell_sp) {
    if (a.w_max <= 1 || atoms <= 1) return 1u;
    const double n_cell = (double)cell_sp / (a.h * a.h * a.h);
    const double r = sqrt(n_cell / a.n_max * (double)atoms);
    const double w = ceil(r > 1.0 ? r : 1.0);
    return w < (double)a.w_max ? (uint32_t)w : (uint32_t)a.w_max;
}

__device__ inline double interp_phi(const Grid& g, const double* phi, double X, double Y, double Z) {
    int i = clampi((int)floor(X), 0, g.nx - 2), j = clampi((int)floor(Y), 0, g.ny - 2),
        k = clampi((int)floor(Z), 0, g.nz - 2);
    double fx = X - i, fy = Y - j, fz = Z - k;
    double s = 0.0;
    for (int t = 0; t < 8; ++t) {
        double w = ((t & 1) ? fx : 1.0 - fx) * ((t & 2) ? fy : 1.0 - fy) * ((t & 4) ? fz : 1.0 - fz);
        int64_t m = ((int64_t)(k + ((t >> 2) & 1)) * g.ny + j + ((t >> 1) & 1)) * g.nx + i + (t & 1);
        s += w * phi[m];
    }
    return s;
}

// point on patch p for uniforms (ua, ub): out = {X, Y, Z, nx, ny, nz, area}
__device__ inline void patch_point(const InjArgs& a, int64_t p, double ua, double ub, double out[7]) {
    const Grid& g = a.g;
    int64_t ring = p / a.naz, az = p % a.naz;
    double ph = 2.0 * kPi * ((double)az + ub) / (double)a.naz;
    double sp, cp;
    sincos(ph, &sp, &cp);
    if (ring < a.rings) {
        double ct = 1.0 - ((double)ring + ua) / (double)a.rings;
        double st = sqrt(1.0 - ct * ct);
        double nx = st * cp, ny = st * sp, nz = ct;
        out[0] = g.xc + g.R * nx;
        out[1] = g.yc + g.R * ny;
        out[2] = g.zc + g.R * nz;
        out[3] = nx;
        out[4] = ny;
        out[5] = nz;
        out[6] = 2.0 * kPi * g.R * g.R / (double)a.rings / (double)a.naz;
    } else {
        int64_t q = ring - a.rings;
        double zlo = (double)q, zhi = fmin((double)(q + 1), g.zc);
        out[0] = g.xc + g.R * cp;
        out[1] = g.yc + g.R * sp;
        out[2] = zlo + ua * (zhi - zlo);
        out[3] = cp;
        out[4] = sp;
        out[5] = 0.0;
        out[6] = 2.0 * kPi * g.R * (zhi - zlo) / (double)a.naz;
    }
}

__device__ inline int64_t patch_count(const InjArgs& a, int64_t p, double* nexp, int* clamped) {
    double q[7];
    patch_point(a, p, 0.5, 0.5, q);
    *clamped = 0;
    if (a.kind == 1) {
        const double N = a.evap_flux * q[6] * a.h * a.h * a.dt;
        *nexp = N;
        Draw2 u = draw2(a.seed, (uint32_t)p, a.step, kTagEvap, 0);
        double fl = floor(N);
        const int64_t atoms = (int64_t)fl + ((u.a < N - fl) ? 1 : 0);
        if (!a.weighted) return atoms;
        // atoms -> superparticles of the rule's weight (the last takes the rest)
        const int ci = clampi((int)floor(q[0] + q[3]), 0, a.g.nx - 2);
        const int cj = clampi((int)floor(q[1] + q[4]), 0, a.g.ny - 2);
        const int ck = clampi((int)floor(q[2] + q[5]), 0, a.g.nz - 2);
        const uint32_t key = cell_key(a.g, ci, cj, ck);
        const uint32_t wp = inject_weight(a, atoms, a.off[key + 1] - a.off[key]);
        a.wk[p] = make_uint2(wp, (uint32_t)min(atoms, (int64_t)0xffffffffLL));
        return (atoms + wp - 1) / wp;
    }
    double F = interp_phi(a.g, a.phi, q[0] + q[3], q[1] + q[4], q[2] + q[5]) / a.h;
    double J = 0.0;
    if (F > 0.0) {
        double f = a.fn_cs2 * F / (a.phi_w * a.phi_w);
        if (f > 1.0) {
            f = 1.0;
            *clamped = 1;
        }
        double lf = log(f);
        double v = 1.0 - f + (f / 6.0) * lf;
        double t = 1.0 + f / 9.0 - (f / 18.0) * lf;
        J = a.fn_a * F * F / (a.phi_w * t * t) * exp(-v * a.fn_b * a.phi_w15 / F);
    }
    double N = J * q[6] * a.h * a.h * a.dt / kQe;
    *nexp = N;
    Draw2 u = draw2(a.seed, (uint32_t)p, a.step, kTagInj, 0);
    double fl = floor(N);
    return (int64_t)fl + ((u.a < N - fl) ? 1 : 0);
}

// Counts of every patch, one patch per thread over many blocks (the work is
// FP64 transcendentals and a gather, too much for one compute unit). A count
// that does not fit 32 bits is stored as 0xffffffff, which overflows any
// buffer. Each block leaves its sums of the expected counts and of the
// clamped patches, added later in block order.
__global__ __launch_bounds__(kInjCountBlock) void k_inject_count(InjArgs a) {
    __shared__ double shd[kInjCountBlock / 64];
    const int64_t p = (int64_t)blockIdx.x * kInjCountBlock + threadIdx.x;
    double ne = 0.0;
    int cl = 0;
    if (p < a.npatch) {
        const int64_t k = patch_count(a, p, &ne, &cl);
        a.cnt[p] = (uint32_t)min(k, (int64_t)0xffffffffLL);
    }
    const double NE = block_sum(ne, shd);
    const double CL = block_sum((double)cl, shd);
    if (threadIdx.x == 0) {
        a.part[2 * blockIdx.x] = NE;
        a.part[2 * blockIdx.x + 1] = CL;
    }
}

// Electrons of the emission, in patch order: one block of 1024 threads over
// chunks of 8192 patches. The chunk's counts go to shared memory and a block
// scan turns them into offsets in patch order (each thread takes a run of 8,
// wavefront shuffles, then the 16 wavefront totals); then the chunk's
// electrons are spread evenly over the threads, each finding its patch by
// binary search over the offsets, so that consecutive electrons go to
// consecutive slots. A chunk that would overflow the buffer sets the capacity
// error; its electrons and those of later chunks are not made, and the
// particle count is left as it was. The expected count takes every patch.
constexpr int kInjBlock = 1024, kInjPer = 8, kInjChunk = kInjBlock * kInjPer;

// exclusive prefix of v over the block and the block total
__device__ inline int64_t inj_scan(int64_t v, int64_t* wsum, int64_t& total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int64_t pre = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < kInjBlock / 64; ++q) {
        const int64_t t = wsum[q];
        pre += q < w ? t : 0;
        tot += t;
    }
    __syncthreads();  // wsum is reused by the next call
    total = tot;
    return pre + x - v;
}

template <typename T>
__global__ __launch_bounds__(kInjBlock) void k_inject(InjArgs a, Species<T> e) {
    __shared__ uint32_t poff[kInjChunk];  // counts, then offsets within the chunk
    __shared__ int64_t wsum[kInjBlock / 64];
    __shared__ double shd[kInjBlock / 64];
    const int t = threadIdx.x;
    const int sp = a.kind == 0 ? PIC_ELECTRON : PIC_NEUTRAL;
    const int64_t base = (int64_t)a.st->n_slots[sp];
    const uint32_t id0 = (uint32_t)a.st->next_id;
    int64_t carry = 0;
    unsigned long long atoms = 0;   // the weights this thread wrote
    bool over = false;
    for (int64_t c0 = 0; c0 < a.npatch; c0 += kInjChunk) {
        bool big = false;
#pragma unroll
        for (int u = 0; u < kInjPer; ++u) {
            const int64_t p = c0 + u * kInjBlock + t;
            const uint32_t k = p < a.npatch ? a.cnt[p] : 0u;
            big |= k == 0xffffffffu;
            poff[u * kInjBlock + t] = k;
        }
        big = __syncthreads_or(big);
        // offsets in patch order
        uint32_t r[kInjPer];
        int64_t run = 0;
#pragma unroll
        for (int u = 0; u < kInjPer; ++u) {
            r[u] = poff[t * kInjPer + u];
            run += r[u];
        }
        int64_t tchunk;
        int64_t o = inj_scan(run, wsum, tchunk);
        over = over || big || base + carry + tchunk > a.cap || tchunk > (int64_t)0xffffffffLL;
        if (!over) {
#pragma unroll
            for (int u = 0; u < kInjPer; ++u) {
                poff[t * kInjPer + u] = (uint32_t)o;
                o += r[u];
            }
        }
        __syncthreads();
        if (!over) {
            for (int64_t q = t; q < tchunk; q += kInjBlock) {
                // the last patch whose offset is <= q (offsets past the chunk's
                // last patch equal the chunk total, which is > q)
                int lo = 0;
#pragma unroll
                for (int s = kInjChunk / 2; s > 0; s >>= 1)
                    if ((int64_t)poff[lo + s] <= q) lo += s;
                const int64_t p = c0 + lo, j = q - (int64_t)poff[lo];
                const int64_t m = base + carry + q;
                double pt[7];
                if (a.kind == 0) {
                    Draw2 d = draw2(a.seed, (uint32_t)p, a.step, kTagInj, (uint32_t)(1 + j));
                    patch_point(a, p, d.a, d.b, pt);
                    e.vx[m] = (T)0;
                    e.vy[m] = (T)0;
                    e.vz[m] = (T)0;
                } else {
                    Draw2 d = draw2(a.seed, (uint32_t)p, a.step, kTagEvap, (uint32_t)(1 + 3 * j));
                    Draw2 w12 = draw2(a.seed, (uint32_t)p, a.step, kTagEvap, (uint32_t)(2 + 3 * j));
                    Draw2 w3 = draw2(a.seed, (uint32_t)p, a.step, kTagEvap, (uint32_t)(3 + 3 * j));
                    patch_point(a, p, d.a, d.b, pt);
                    // outward normal n and the tangents t1 = (-n_y, n_x, 0) / |.|, t2 = n x t1
                    const double n0 = pt[3], n1 = pt[4], n2 = pt[5];
                    const double tl = sqrt(n0 * n0 + n1 * n1);
                    const double t10 = -n1 / tl, t11 = n0 / tl, t12 = 0.0;
                    const double t20 = n1 * t12 - n2 * t11, t21 = n2 * t10 - n0 * t12, t22 = n0 * t11 - n1 * t10;
                    const double vn = a.vsig * sqrt(-2.0 * log(w12.a));
                    const double rt = a.vsig * sqrt(-2.0 * log(w12.b));
                    double sn, cs;
                    sincos(2.0 * kPi * w3.a, &sn, &cs);
                    const double va = rt * cs, vb = rt * sn;
                    e.vx[m] = (T)(vn * n0 + va * t10 + vb * t20);
                    e.vy[m] = (T)(vn * n1 + va * t11 + vb * t21);
                    e.vz[m] = (T)(vn * n2 + va * t12 + vb * t22);
                }
                e.x[m] = (T)(pt[0] + 1e-3 * pt[3]);
                e.y[m] = (T)(pt[1] + 1e-3 * pt[4]);
                e.z[m] = (T)(pt[2] + 1e-3 * pt[5]);
                e.id[m] = id0 + (uint32_t)(carry + q);
                if (e.w) {
                    uint32_t wgt = 1u;
                    if (a.kind == 1) {
                        const uint2 wk = a.wk[p];
                        const int64_t k = ((int64_t)wk.y + wk.x - 1) / wk.x;
                        wgt = j + 1 < k ? wk.x : (uint32_t)((int64_t)wk.y - (k - 1) * (int64_t)wk.x);
                    }
                    e.w[m] = wgt;
                    atoms += wgt;
                } else {
                    atoms += 1;
                }
            }
        }
        carry += tchunk;
        __syncthreads();  // poff is rewritten by the next chunk
    }
    // the count blocks' sums, in block order
    const int64_t nb = (a.npatch + kInjCountBlock - 1) / kInjCountBlock;
    double ne = 0.0, cl = 0.0;
    for (int64_t b = t; b < nb; b += kInjBlock) {
        ne += a.part[2 * b];
        cl += a.part[2 * b + 1];
    }
    const double NE = block_sum(ne, shd);
    const double CL = block_sum(cl, shd);
    __shared__ unsigned long long shu[kInjBlock / 64];
    const unsigned long long AT = block_sum(atoms, shu);
    if (t == 0) {
        if (a.kind == 0) {
            a.st->fn_expected += NE;
            a.st->fn_clamped += (unsigned long long)CL;
        } else {
            a.st->evap_expected += NE;
        }
        if (over) {
            atomicCAS(&a.st->error, 0, PIC_E_CAPACITY);
        } else {
            a.st->n_slots[sp] += (unsigned long long)carry;
            a.st->next_id += (unsigned long long)carry;
            if (a.kind == 0) {
                a.st->injected += (unsigned long long)carry;
            } else {
                a.st->evaporated += (unsigned long long)carry;
                a.st->evap_atoms += AT;
            }
        }
    }
}

hipError_t inject_phase(pic_ctx* c) { return inject_phase_in(c, c->inj_cnt, c->inj_part); }

// cnt: npatch uint32 counts; part: 2 doubles per count block. Every entry the
// emission reads is written earlier in the same call, so neither needs
// clearing.
hipError_t inject_phase_in(pic_ctx* c, uint32_t* cnt, double* part) {
    InjArgs a;
    a.g = c->g;
    a.phi = c->buf.phi;
    a.rings = c->cfg.fn_rings;
    a.naz = c->cfg.fn_az;
    a.npatch = c->npatch;
    a.fn_a = kQe * kQe / (8.0 * kPi * kHpl);
    a.fn_b = (8.0 * kPi / 3.0) * sqrt(2.0 * kMe) / (kQe * kHpl) * pow(kQe, 1.5);
    a.fn_cs2 = kQe / (4.0 * kPi * kEps0);
    a.phi_w = c->cfg.phi_w;
    a.h = c->cfg.h;
    a.dt = c->cfg.dt;
    a.seed = c->cfg.seed;
    a.step = (uint32_t)c->step;
    a.st = c->st;
    a.cap = c->buf.cap[0];
    a.phi_w15 = pow(a.phi_w, 1.5);
    a.cnt = cnt;
    a.part = part;
    a.kind = 0;
    a.evap_flux = 0.0;
    a.vsig = 0.0;
    a.weighted = c->cfg.weighted;
    a.w_max = c->cfg.w_max;
    a.n_max = c->cfg.n_max;
    a.off = c->off;
    a.wk = (uint2*)(part + 2 * ((c->npatch + kInjCountBlock - 1) / kInjCountBlock));
    if (c->npatch == 0) return hipSuccess;
    const int64_t nb = (c->npatch + kInjCountBlock - 1) / kInjCountBlock;
    // field emission, then (same work memory, in stream order) evaporation
    for (int kind = 0; kind < 2; ++kind) {
        if (kind == 1) {
            if (!(c->cfg.surface_T > 0.0)) break;
            a.kind = 1;
            a.evap_flux = c->evap_flux;
            a.vsig = c->evap_vsig;
            a.cap = c->buf.cap[PIC_NEUTRAL];
        }
        const int sp = kind == 0 ? PIC_ELECTRON : PIC_NEUTRAL;
        hipLaunchKernelGGL(k_inject_count, dim3((unsigned)nb), dim3(kInjCountBlock), 0, c->stream, a);
        if (c->cfg.precision == PIC_F32)
            hipLaunchKernelGGL(k_inject<float>, dim3(1), dim3(kInjBlock), 0, c->stream, a, species<float>(c, sp));
        else
            hipLaunchKernelGGL(k_inject<double>, dim3(1), dim3(kInjBlock), 0, c->stream, a, species<double>(c, sp));
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Explicit load: append n particles, numbered from next_id in array order.

template <typename T>
__global__ void k_load(Species<T> s, int sp, const T* x, const T* y, const T* z, const T* vx, const T* vy,
                       const T* vz, const uint32_t* w, int64_t n, DevState* st) {
    int64_t base = (int64_t)st->n_slots[sp];
    if (base + n > s.cap) return;
    uint32_t id0 = (uint32_t)st->next_id;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        int64_t m = base + i;
        s.x[m] = x[i];
        s.y[m] = y[i];
        s.z[m] = z[i];
        s.vx[m] = vx[i];
        s.vy[m] = vy[i];
        s.vz[m] = vz[i];
        s.id[m] = id0 + (uint32_t)i;
        if (s.w) s.w[m] = w ? w[i] : 1u;
    }
}

__global__ void k_load_finish(DevState* st, int sp, int64_t n, int64_t cap) {
    if ((int64_t)st->n_slots[sp] + n > cap) {
        atomicCAS(&st->error, 0, PIC_E_CAPACITY);
        return;
    }
    st->n_slots[sp] += (unsigned long long)n;
    st->next_id += (unsigned long long)n;
}

hipError_t load_particles(pic_ctx* c, const pic_particles* src) {
    int s = src->species;
    if (src->n == 0) return hipSuccess;
    if (c->cfg.precision == PIC_F32) {
        hipLaunchKernelGGL(k_load<float>, dim3(grid_for(src->n)), dim3(kBlock), 0, c->stream, species<float>(c, s), s,
                           (const float*)src->x, (const float*)src->y, (const float*)src->z, (const float*)src->vx,
                           (const float*)src->vy, (const float*)src->vz, src->w, src->n, c->st);
    } else {
        hipLaunchKernelGGL(k_load<double>, dim3(grid_for(src->n)), dim3(kBlock), 0, c->stream, species<double>(c, s),
                           s, (const double*)src->x, (const double*)src->y, (const double*)src->z,
                           (const double*)src->vx, (const double*)src->vy, (const double*)src->vz, src->w, src->n,
                           c->st);
    }
    hipLaunchKernelGGL(k_load_finish, dim3(1), dim3(1), 0, c->stream, c->st, s, src->n, c->buf.cap[s]);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Moments: per species the alive count and kinetic energy, and the
// Shockley-Ramo current I = sum q v . E0(x) (Sec. 2.3.1) with E0 the field of
// the unit-anode Laplace problem. Fixed grid and fixed-order reductions.
// out (device, per block): 10 doubles {n_e, n_i, n_n, ke_e, ke_i, ke_n, i_sr,
// and the physical counts (sums of the weights) of the three species}.
constexpr int kMomVals = 10;

constexpr int kMomBlocks = 512;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_moments(Species<T> s0, Species<T> s1, Species<T> s2,
                                                     const typename V4<T>::type* E0, Grid g, double sv, double m_ion,
                                                     const DevState* st, double* part, const int64_t* rho,
                                                     long long* qpart) {
    __shared__ double sh[kBlock / 64];
    double acc[kMomVals] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const Species<T>* S[3] = {&s0, &s1, &s2};
    const double mass[3] = {kMe, m_ion, m_ion};
    const double q[3] = {-kQe, kQe, 0.0};
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int s = 0; s < 3; ++s) {
        int64_t n = (int64_t)st->n_slots[s];
        const Species<T>& P = *S[s];
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
            if (P.id[i] == kDead) continue;
            double vx = (double)P.vx[i] * sv, vy = (double)P.vy[i] * sv, vz = (double)P.vz[i] * sv;
            const double wp = P.w ? (double)P.w[i] : 1.0;
            acc[s] += 1.0;
            acc[7 + s] += wp;
            acc[3 + s] += wp * 0.5 * mass[s] * (vx * vx + vy * vy + vz * vz);
            if (s != 2) {
                T ex, ey, ez;
                gather<T>(g, E0, P.x[i], P.y[i], P.z[i], ex, ey, ez);
                acc[6] += wp * q[s] * (vx * (double)ex + vy * (double)ey + vz * (double)ez);
            }
        }
    }
    for (int k = 0; k < kMomVals; ++k) {
        double t = block_sum(acc[k], sh);
        if (threadIdx.x == 0) part[blockIdx.x * kMomVals + k] = t;
    }
    long long qs = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.nn; i += stride) qs += rho[i];
    __shared__ long long shl[kBlock / 64];
    long long tq = block_sum(qs, shl);
    if (threadIdx.x == 0) qpart[blockIdx.x] = tq;
}

// out: the 7 sums, the total charge (int64 in out[7]), the 3 physical counts
__global__ void k_moments_final(const double* part, int nb, const long long* qpart, double* out) {
    __shared__ double sh[kBlock / 64];
    for (int k = 0; k < kMomVals; ++k) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[b * kMomVals + k];
        double t = block_sum(s, sh);
        if (threadIdx.x == 0) out[k < 7 ? k : k + 1] = t;
    }
    __shared__ long long shl[kBlock / 64];
    long long q = 0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) q += qpart[b];
    long long tq = block_sum(q, shl);
    if (threadIdx.x == 0) ((long long*)out)[7] = tq;
}

hipError_t moments_phase(pic_ctx* c, double* out_dev) {
    double sv = c->cfg.h / c->cfg.dt;
    double* part = c->partials;
    if (c->cfg.precision == PIC_F32)
        hipLaunchKernelGGL(k_moments<float>, dim3(kMomBlocks), dim3(kBlock), 0, c->stream, species<float>(c, 0),
                           species<float>(c, 1), species<float>(c, 2), (const float4*)c->buf.field0, c->g, sv,
                           c->cfg.m_ion, c->st, part, c->buf.rho, (long long*)(part + kMomVals * kMomBlocks));
    else
        hipLaunchKernelGGL(k_moments<double>, dim3(kMomBlocks), dim3(kBlock), 0, c->stream, species<double>(c, 0),
                           species<double>(c, 1), species<double>(c, 2), (const double4*)c->buf.field0, c->g, sv,
                           c->cfg.m_ion, c->st, part, c->buf.rho, (long long*)(part + kMomVals * kMomBlocks));
    hipLaunchKernelGGL(k_moments_final, dim3(1), dim3(kBlock), 0, c->stream, part, kMomBlocks,
                       (const long long*)(part + kMomVals * kMomBlocks), out_dev);
    return hipGetLastError();
}

}  // namespace pic
