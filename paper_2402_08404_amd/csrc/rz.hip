// rz.hip -- the 2D axisymmetric (r, z) 2D3V variant of the particle-mesh
// step (Sec. 2.2): node types of the axisymmetric tip, Poisson's equation in
// cylindrical finite-volume form by FP64 conjugate gradients, the node
// field, gather + leapfrog push with the rotation back into the r-z plane,
// removal, and the fixed-point deposit. The discretization is stated in
// pic_rz.h.
#include <algorithm>
#include <cmath>
#include <string>

#include "pic_internal.hpp"
#include "pic_rz.h"

namespace pic_rz {

using pic::clampi;
using pic::kBlock;
using pic::kDead;
using pic::kEps0;
using pic::kMe;
using pic::kPi;
using pic::kQe;

constexpr int kCgBlocks = 256;  // blocks of the CG kernels (one partial each, summed in block order)
constexpr uint8_t kFree = 0, kHeld0 = 1, kHeldV = 2;  // node types

struct State {
    unsigned long long absorbed[3][5];
    double rr, bb, pq, alpha, beta, rtol;
    int it, maxit, done, error;
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

__global__ void k_types(Geo g, uint8_t* type) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (int64_t)g.nr * g.nz) return;
    const int i = (int)(n % g.nr), k = (int)(n / g.nr);
    uint8_t t = kFree;
    if (inside_tip(g, (double)i, (double)k)) t = kHeld0;
    if (k == 0) t = kHeld0;
    if (k == g.nz - 1) t = kHeldV;
    type[n] = t;
}

// sum_j c (x_n - x_m) at a free node n (x of held neighbours as given)
__device__ inline double apply_at(const Geo& g, const double* x, int64_t n) {
    const int i = (int)(n % g.nr);
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
    double *r, *p, *q;
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

// phi at held nodes to their values; r = b - A phi and p = r on free nodes;
// partials of r.r and of the right-hand side with the held values moved over
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
        const int i = (int)(n % a.g.nr);
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
        a.p[n] = r;
        rr += r * r;
        const double be = b + lift;
        bb += be * be;
    }
    block_reduce2(rr, bb, a.part);
}

// (single block) rr, bb from the partials
__global__ void k_cg_start(CgArgs a, double rtol, int maxit) {
    if (threadIdx.x == 0) {
        double rr = 0.0, bb = 0.0;
        for (int b = 0; b < kCgBlocks; ++b) {
            rr += a.part[2 * b];
            bb += a.part[2 * b + 1];
        }
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
    if (threadIdx.x == 0) {
        double pq = 0.0;
        for (int b = 0; b < kCgBlocks; ++b) pq += a.part[2 * b];
        alpha = a.st->rr / pq;
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

// (single block) beta, convergence
__global__ void k_cg_scalars(CgArgs a) {
    if (threadIdx.x != 0) return;
    State* st = a.st;
    if (st->done) return;
    double rr = 0.0;
    for (int b = 0; b < kCgBlocks; ++b) rr += a.part[2 * kCgBlocks + 2 * b];
    st->beta = rr / st->rr;
    st->rr = rr;
    st->it += 1;
    if (rr <= st->rtol * st->rtol * st->bb || st->it >= st->maxit) st->done = 1;
}

__global__ __launch_bounds__(kBlock) void k_cg_p(CgArgs a) {
    if (a.st->done) return;
    const double beta = a.st->beta;
    const int64_t nn = (int64_t)a.g.nr * a.g.nz;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += (int64_t)gridDim.x * blockDim.x)
        if (a.type[n] == kFree) a.p[n] = a.r[n] + beta * a.p[n];
}

__global__ void k_field(Geo g, const double* phi, double h, double* E) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (int64_t)g.nr * g.nz) return;
    const int i = (int)(n % g.nr), k = (int)(n / g.nr);
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
    int64_t n;
    const double* E;
    double kq;  // (q / m) dt^2 / h
    int sp;
    State* st;
};

__global__ __launch_bounds__(kBlock) void k_push(PushArgs a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n || a.id[p] == kDead) return;
    const Geo& g = a.g;
    double r = a.r[p], z = a.z[p], vr = a.vr[p], vt = a.vt[p], vz = a.vz[p];
    if (a.kq != 0.0) {
        const int i = clampi((int)floor(r), 0, g.nr - 2), k = clampi((int)floor(z), 0, g.nz - 2);
        const double fr = r - i, fz = z - k;
        const int64_t n0 = (int64_t)k * g.nr + i;
        const double w00 = (1 - fr) * (1 - fz), w10 = fr * (1 - fz), w01 = (1 - fr) * fz, w11 = fr * fz;
        const double er = w00 * a.E[2 * n0] + w10 * a.E[2 * (n0 + 1)] + w01 * a.E[2 * (n0 + g.nr)] +
                          w11 * a.E[2 * (n0 + g.nr + 1)];
        const double ez = w00 * a.E[2 * n0 + 1] + w10 * a.E[2 * (n0 + 1) + 1] + w01 * a.E[2 * (n0 + g.nr) + 1] +
                          w11 * a.E[2 * (n0 + g.nr + 1) + 1];
        vr += a.kq * er;
        vz += a.kq * ez;
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

__global__ __launch_bounds__(kBlock) void k_deposit(Geo g, const double* r, const double* z, const uint32_t* id,
                                                     int64_t n, int64_t sign, int64_t* rho) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n || id[p] == kDead) return;
    const double R = r[p], Z = z[p];
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

__global__ void k_counts(const uint32_t* id, int64_t n, unsigned long long* out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool alive = p < n && id[p] != kDead;
    const unsigned long long m = __ballot(alive);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(out, (unsigned long long)__popcll(m));
}

__global__ void k_qsum(const int64_t* rho, int64_t nn, unsigned long long* out) {
    long long s = 0;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += (int64_t)gridDim.x * blockDim.x)
        s += rho[n];
    s = pic::wave_sum(s);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(out, (unsigned long long)s);
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// scratch: State, CG vectors r, p, q, partials (4 * kCgBlocks), counters (8)
size_t layout(const pic_rz_config* c, char* base, State** st, double** r, double** p, double** q, double** part,
              unsigned long long** cnt) {
    const size_t nn = (size_t)c->nr * c->nz;
    size_t off = 0;
    auto take = [&](size_t b) -> char* {
        char* x = base ? base + off : nullptr;
        off = align256(off + b);
        return x;
    };
    char* a = take(sizeof(State));
    char* b = take(nn * 8);
    char* d = take(nn * 8);
    char* e = take(nn * 8);
    char* f = take(4 * kCgBlocks * 8);
    char* g = take(8 * 8);
    if (st) *st = (State*)a;
    if (r) *r = (double*)b;
    if (p) *p = (double*)d;
    if (q) *q = (double*)e;
    if (part) *part = (double*)f;
    if (cnt) *cnt = (unsigned long long*)g;
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
    return nullptr;
}

}  // namespace pic_rz

struct pic_rz_ctx {
    pic_rz_config cfg;
    pic_rz_buffers buf;
    hipStream_t stream = nullptr;
    pic_rz::Geo g;
    pic_rz::State* st = nullptr;
    double *r = nullptr, *p = nullptr, *q = nullptr, *part = nullptr;
    unsigned long long* cnt = nullptr;
    double V0 = 0.0, F1 = 0.0;
    int64_t step = 0;
    int last_iters = 0;
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
    a.part = c->part;
    a.st = c->st;
    a.qscale = std::ldexp(1.0, -40) * kQe / (kPi * kEps0 * c->cfg.h);
    a.V0 = V0;
    return a;
}

// CG from the current phi (held nodes set to 0 / V0); without charge the
// q vector, zeroed, stands for the charge (it is read only by k_cg_init,
// before the iterations use q)
pic_status cg(pic_rz_ctx* c, double* phi, double V0, bool with_charge, double rtol, int maxit, int* iters) {
    CgArgs a = cg_args(c, phi, V0);
    if (!with_charge) {
        pic_status s = hip_ok(c, hipMemsetAsync(c->q, 0, (size_t)c->g.nr * c->g.nz * 8, c->stream), "zero");
        if (s != PIC_OK) return s;
        a.rho = (const int64_t*)c->q;
    }
    hipLaunchKernelGGL(k_cg_init, dim3(kCgBlocks), dim3(kBlock), 0, c->stream, a);
    hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(64), 0, c->stream, a, rtol, maxit);
    State h{};
    for (;;) {
        for (int k = 0; k < 16; ++k) {
            hipLaunchKernelGGL(k_cg_ap, dim3(kCgBlocks), dim3(kBlock), 0, c->stream, a);
            hipLaunchKernelGGL(k_cg_update, dim3(kCgBlocks), dim3(kBlock), 0, c->stream, a);
            hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(64), 0, c->stream, a);
            hipLaunchKernelGGL(k_cg_p, dim3(kCgBlocks), dim3(kBlock), 0, c->stream, a);
        }
        pic_status s = hip_ok(c, hipMemcpyAsync(&h, c->st, sizeof(State), hipMemcpyDeviceToHost, c->stream), "copy");
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

}  // namespace

extern "C" {

pic_status pic_rz_scratch_size(const pic_rz_config* cfg, const int64_t cap[3], size_t* bytes) {
    if (check(cfg) || !cap || !bytes) return PIC_E_INVALID_ARG;
    *bytes = layout(cfg, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    return PIC_OK;
}

pic_status pic_rz_init(const pic_rz_config* cfg, const pic_rz_buffers* bufs, void* hip_stream, pic_rz_ctx** out) {
    if (!out) return PIC_E_INVALID_ARG;
    *out = nullptr;
    if (check(cfg) || !bufs) return PIC_E_INVALID_ARG;
    if (!bufs->phi || !bufs->phi1 || !bufs->rho || !bufs->field || !bufs->node_type || !bufs->scratch)
        return PIC_E_INVALID_ARG;
    if (bufs->scratch_bytes < layout(cfg, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr))
        return PIC_E_INVALID_ARG;
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
    layout(cfg, base, &c->st, &c->r, &c->p, &c->q, &c->part, &c->cnt);
    const int64_t nn = (int64_t)cfg->nr * cfg->nz;
    pic_status s = hip_ok(c, hipMemsetAsync(c->st, 0, sizeof(State), c->stream), "zero");
    if (s == PIC_OK) {
        hipLaunchKernelGGL(k_types, dim3(grid_of(nn)), dim3(kBlock), 0, c->stream, c->g, bufs->node_type);
        s = hip_ok(c, hipMemsetAsync(bufs->phi1, 0, nn * 8, c->stream), "zero");
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
    const double qm[3] = {-kQe / kMe, kQe / c->cfg.m_ion, 0.0};
    for (int t = 0; t < nsteps; ++t) {
        if (flags & PIC_RZ_PUSH) {
            for (int s = 0; s < 3; ++s) {
                if (c->buf.n[s] == 0) continue;
                PushArgs a;
                a.g = c->g;
                a.r = c->buf.r[s];
                a.z = c->buf.z[s];
                a.vr = c->buf.vr[s];
                a.vt = c->buf.vt[s];
                a.vz = c->buf.vz[s];
                a.id = c->buf.id[s];
                a.n = c->buf.n[s];
                a.E = c->buf.field;
                a.kq = qm[s] * c->cfg.dt * c->cfg.dt / c->cfg.h;
                a.sp = s;
                a.st = c->st;
                hipLaunchKernelGGL(k_push, dim3(grid_of(a.n)), dim3(kBlock), 0, c->stream, a);
            }
        }
        if (flags & PIC_RZ_DEPOSIT) {
            const int64_t nn = (int64_t)c->g.nr * c->g.nz;
            hipLaunchKernelGGL(k_zero_rho, dim3(grid_of(nn)), dim3(kBlock), 0, c->stream, c->buf.rho, nn);
            for (int s = 0; s < 2; ++s)
                if (c->buf.n[s] > 0)
                    hipLaunchKernelGGL(k_deposit, dim3(grid_of(c->buf.n[s])), dim3(kBlock), 0, c->stream, c->g,
                                       c->buf.r[s], c->buf.z[s], c->buf.id[s], c->buf.n[s], s == 0 ? -1 : 1,
                                       c->buf.rho);
        }
        pic_status st = hip_ok(c, hipGetLastError(), "step");
        if (st != PIC_OK) return st;
        if (flags & PIC_RZ_SOLVE) {
            st = pic_rz_solve(c, c->cfg.step_rtol, c->cfg.maxit, nullptr);
            if (st != PIC_OK) return st;
        } else if (flags & PIC_RZ_FIELD) {
            st = field(c);
            if (st != PIC_OK) return st;
        }
        if (flags & PIC_RZ_ADVANCE) c->step++;
    }
    return PIC_OK;
}

pic_status pic_rz_moments(pic_rz_ctx* c, pic_rz_moments_t* out) {
    if (!c || !out) return PIC_E_INVALID_ARG;
    pic_status s = hip_ok(c, hipMemsetAsync(c->cnt, 0, 8 * 8, c->stream), "zero");
    if (s != PIC_OK) return s;
    for (int sp = 0; sp < 3; ++sp)
        if (c->buf.n[sp] > 0)
            hipLaunchKernelGGL(k_counts, dim3(grid_of(c->buf.n[sp])), dim3(kBlock), 0, c->stream, c->buf.id[sp],
                               c->buf.n[sp], c->cnt + sp);
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
    return PIC_OK;
}

const char* pic_rz_last_error(const pic_rz_ctx* c) { return c ? c->err.c_str() : "no context"; }

void pic_rz_destroy(pic_rz_ctx* c) { delete c; }

}  // extern "C"
