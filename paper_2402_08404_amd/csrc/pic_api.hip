// pic_api.hip -- the extern "C" entry points declared in include/pic.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "pic_internal.hpp"

using namespace pic;

// Work memory of pic_inject_noalloc: a static device array, one copy per GPU
// for the life of the process. In host code its name is not a device
// address; the address of each device's copy is taken once per device with
// hipGetSymbolAddress (static_work_setup, called by pic_init) and only that
// address is used.
constexpr size_t kStaticWorkBytes = (size_t)1 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticWorkBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_addr[kMaxDevices] = {};

// The address of the current device's copy of the static work array.
hipError_t static_work_setup(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_static_addr[dev] = p;
    }
    *out = g_static_addr[dev];
    return hipSuccess;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

pic_status fail(pic_ctx* c, pic_status code, const std::string& msg) {
    if (c) {
        c->err = msg;
        if (code == PIC_E_HIP || code == PIC_E_CAPACITY || code == PIC_E_OVERFLOW) c->failed = code;
    }
    return code;
}

pic_status hip_check(pic_ctx* c, hipError_t e, const char* where) {
    if (e == hipSuccess) return PIC_OK;
    return fail(c, PIC_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

double adk_rate(double c, double e, double x32, double E) {
    return c * std::pow(20.5 * x32 / E, e) * std::exp(-6.83 * x32 / E);
}

// Groups of the binning: 2^s consecutive tiles with s the smallest that
// leaves at most kBinTargetGroups groups, but no group above
// kBinMaxCellsPerGroup cells; false if that leaves more than kBinMaxGroups.
bool bin_groups(int64_t ntiles, int* ng, int* gshift) {
    int sh = 0;
    while (((ntiles + (1 << sh) - 1) >> sh) > kBinTargetGroups && (kTileCells << (sh + 1)) <= kBinMaxCellsPerGroup)
        ++sh;
    *ng = (int)((ntiles + (1 << sh) - 1) >> sh);
    *gshift = 9 + sh;
    return *ng <= kBinMaxGroups;
}

const char* check_config(const pic_config* cfg) {
    if (!cfg) return "config is NULL";
    if (cfg->nx < 4 || cfg->ny < 4 || cfg->nz < 4) return "nx, ny, nz must be >= 4";
    if ((int64_t)cfg->nx * cfg->ny * cfg->nz >= (int64_t)1 << 31) return "grid too large";
    {
        const int64_t ntiles =
            (int64_t)((cfg->nx - 2) / kTile + 1) * ((cfg->ny - 2) / kTile + 1) * ((cfg->nz - 2) / kTile + 1);
        int ng = 0, gshift = 0;
        if (!bin_groups(ntiles, &ng, &gshift))
            return "grid too large for the cell binning (over 131072 tiles of 8^3 cells)";
    }
    if (!(cfg->h > 0) || !(cfg->dt > 0)) return "h and dt must be positive";
    if (!(cfg->tip_r > 0) || !(cfg->tip_h >= cfg->tip_r)) return "need tip_r > 0 and tip_h >= tip_r";
    double R = cfg->tip_r / cfg->h, H = cfg->tip_h / cfg->h;
    if (R + 2.0 >= 0.5 * (cfg->nx - 1) || R + 2.0 >= 0.5 * (cfg->ny - 1) || H + 2.0 >= cfg->nz - 1)
        return "the tip does not fit in the box with two spacings to spare";
    if (cfg->precision != PIC_F64 && cfg->precision != PIC_F32) return "precision must be PIC_F64 or PIC_F32";
    if (cfg->solver < PIC_SOLVER_CG || cfg->solver > PIC_SOLVER_MIXED) return "unknown solver";
    if (cfg->xs_n < 2 || !cfg->xs_el || !cfg->xs_iz || !cfg->xs_cx) return "need three tables of >= 2 entries";
    if (!(cfg->xs_emin > 0) || !(cfg->xs_emax > cfg->xs_emin)) return "need 0 < xs_emin < xs_emax";
    for (int k = 0; k < cfg->xs_n; ++k)
        if (!(cfg->xs_el[k] >= 0) || !(cfg->xs_iz[k] >= 0) || !(cfg->xs_cx[k] >= 0))
            return "cross sections must be finite and >= 0";
    if (cfg->fn_rings < 0 || cfg->fn_az < 0 || (cfg->fn_rings > 0) != (cfg->fn_az > 0))
        return "fn_rings and fn_az must both be positive (or both 0: no emission)";
    if (!(cfg->phi_w > 0) || !(cfg->xi > 0) || !(cfg->m_ion > 0)) return "phi_w, xi, m_ion must be positive";
    if (!(cfg->laplace_rtol > 0) || !(cfg->step_rtol > 0) || cfg->step_maxit < 1) return "bad solver tolerances";
    if (cfg->sort_every < 0) return "sort_every must be >= 0";
    if (cfg->stencil_blocks != 0 && (cfg->stencil_blocks < 64 || cfg->stencil_blocks > 4096))
        return "stencil_blocks must be 0 or in 64..4096";
    if (cfg->step_guess < 0 || cfg->step_guess > 1) return "step_guess must be 0 or 1";
    if (cfg->id_capacity < 0 || cfg->id_capacity > ((int64_t)1 << 32)) return "id_capacity out of range";
    if (!(cfg->surface_T >= 0.0) || !std::isfinite(cfg->surface_T)) return "surface_T must be finite and >= 0";
    if (!(cfg->circuit_R >= 0.0) || !std::isfinite(cfg->circuit_R)) return "circuit_R must be finite and >= 0";
    if (cfg->circuit_R > 0.0 && !(cfg->circuit_C > 0.0 && std::isfinite(cfg->circuit_C)))
        return "the circuit needs circuit_C > 0";
    if (cfg->surface_T > 0.0 && cfg->fn_rings == 0) return "evaporation needs the surface patches (fn_rings, fn_az)";
    if (cfg->weighted != 0 && cfg->weighted != 1) return "weighted must be 0 or 1";
    if (cfg->weighted && cfg->w_max > 1 && !(cfg->n_max > 0.0)) return "the injection weight rule needs n_max > 0";
    if (cfg->merge_every < 0) return "merge_every must be >= 0";
    if (cfg->merge_every > 0 && !cfg->weighted) return "merging needs weighted = 1";
    if (cfg->merge_every > 0 && cfg->merge_max < 1) return "merging needs merge_max >= 1";
    if (cfg->same_species < 0 || cfg->same_species > 7) return "same_species must be 0 .. 7";
    if ((cfg->same_species & 4) && !(cfg->sigma_rec >= 0.0)) return "sigma_rec must be >= 0";
    if (cfg->same_species && cfg->weighted) return "same-species and Coulomb pairing need weighted = 0";
    if ((cfg->same_species & 1) && !(cfg->sigma_nn >= 0.0)) return "sigma_nn must be >= 0";
    if ((cfg->same_species & 2) && !(cfg->coulomb_log > 0.0)) return "coulomb_log must be > 0";
    return nullptr;
}

int64_t id_capacity(const pic_config* cfg, const int64_t cap[3]) {
    if (cfg->id_capacity > 0) return cfg->id_capacity;
    int64_t v = 8 * (cap[0] + cap[1] + cap[2]) + (1 << 20);
    return std::min<int64_t>(v, (int64_t)1 << 32);
}

__global__ void k_scale(double* y, const double* x, double a, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i];
}

__global__ void k_init_state(DevState* st) {
    memset(st, 0, sizeof(DevState));
}

__global__ void k_set_vgap(DevState* st, double v) { st->v_gap = v; }

// Clausius-Clapeyron evaporation flux [1/(m^2 s)] of Cu at T (Sec. 2.3.1):
// p_atm / sqrt(2 pi m k_B T) exp[(E_vap / k_B)(1/T_b - 1/T)], E_vap = 3.43 eV,
// T_b = 2835 K (the boiling point of Cu), p_atm = 101325 Pa.
double evaporation_flux(double m, double T) {
    const double kB = 1.380649e-23, p_atm = 101325.0, e_vap = 3.43, t_boil = 2835.0;
    if (!(T > 0.0)) return 0.0;
    return p_atm / std::sqrt(2.0 * kPi * m * kB * T) * std::exp(e_vap * kQe / kB * (1.0 / t_boil - 1.0 / T));
}

}  // namespace

size_t pic::scratch_layout(pic_ctx* c, const pic_config* cfg, const int64_t cap[3], char* base) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        void* p = base ? (void*)(base + off) : nullptr;
        off = align256(off + bytes);
        return p;
    };
    int64_t nn = (int64_t)cfg->nx * cfg->ny * cfg->nz;
    int64_t ntiles = (int64_t)((cfg->nx - 2) / kTile + 1) * ((cfg->ny - 2) / kTile + 1) * ((cfg->nz - 2) / kTile + 1);
    int64_t nc = ntiles * kTileCells;  // cell keys (tile-major numbering)
    int64_t capsum = cap[0] + cap[1] + cap[2];
    int64_t capmax = std::max(cap[0], std::max(cap[1], cap[2]));
    int64_t idc = id_capacity(cfg, cap);
    int64_t words = (idc + 31) / 32;
    size_t tsz = cfg->precision == PIC_F32 ? 4 : 8;
    int64_t scan_n = std::max(std::max(nc + 1, 256 * ((capsum + 4095) / 4096 + 1)), std::max(capsum, words));
    int64_t scan_blocks = (scan_n + 4095) / 4096 + 1;
    int64_t parts = std::max<int64_t>(4 * 4096, 8 * 512) + 64;  // CG/MG partials (4 x 4096), moments (8 x 512)
    pic_ctx dummy;
    pic_ctx* t = c ? c : &dummy;
    t->st = (DevState*)take(sizeof(DevState));
    t->dyn = (uint32_t*)take(64 * sizeof(uint32_t));
    t->id_ptrs = (uint32_t**)take(3 * sizeof(uint32_t*));
    t->mom_out = (double*)take(16 * sizeof(double));
    t->xs = (double*)take(5 * (size_t)cfg->xs_n * sizeof(double));  // el, iz, cx, rate bounds of the two classes
    t->off = (uint32_t*)take((nc + 1) * 4);
    for (int s = 0; s < 3; ++s) t->key[s] = (uint32_t*)take(cap[s] * 4);
    t->bins = (uint2*)take(capsum * 8);
    t->big = (uint32_t*)take(nc * 4);
    t->mcc_list = (uint32_t*)take(nc * 4);
    t->mcc_count = (uint32_t*)take(4 * 8192 * 4);
    t->mcc_dense = (uint32_t*)take(nc * 4);
    t->fi_list = (uint32_t*)take(cap[2] * 4);
    t->push_part = (uint32_t*)take(8192 * 8 * 4);
    t->push_dpart = (double*)take(8192 * 4 * 8);
    const int64_t npatch = fn_patches(cfg);
    t->inj_cnt = (uint32_t*)take(std::max<int64_t>(npatch, 1) * 4);
    // per count block two doubles, then a {weight, atoms} pair per patch
    t->inj_part = (double*)take(2 * std::max<int64_t>((npatch + kInjCountBlock - 1) / kInjCountBlock, 1) * 8 +
                                std::max<int64_t>(npatch, 1) * 8);
    t->nflag = (uint32_t*)take(cap[2] * 4);
    t->prod_list = (uint32_t*)take(cap[2] * 4);
    t->prod_ev = (int32_t*)take(cap[2] * 4);
    t->prod_ve = (double*)take(cap[2] * 3 * 8);
    for (int k = 0; k < 2; ++k) {
        t->bitmap[k] = (uint32_t*)take(words * 4);
        t->bm_prefix[k] = (uint32_t*)take(words * 4);
    }
    t->ev = (pic_event*)take(cap[2] * sizeof(pic_event));
    t->scan_blocks = (uint32_t*)take(scan_blocks * 4);
    t->rank_flag = (uint32_t*)take(capsum * 4);
    t->rank = (uint32_t*)take(capsum * 4);
    {
        int ng = 1, gshift = 9;
        bin_groups(ntiles, &ng, &gshift);
        int64_t nchunk = 0;
        for (int s = 0; s < 3; ++s) nchunk += (cap[s] + kBinChunk - 1) / kBinChunk;
        t->bin_hist = (uint32_t*)take(std::max<int64_t>(nchunk, 1) * ng * 4);
        t->bin_segtot = (uint32_t*)take((int64_t)kBinSegments * ng * 4);
        t->bin_gbase = (uint32_t*)take(((int64_t)ng + 1) * 4);
        t->bin_stage = (uint4*)take(capsum * 16);
        t->bin_ng = ng;
        t->bin_gshift = gshift;
    }
    t->tmp = take(capmax * (6 * tsz + 8));  // six state arrays, ids, weights
    t->cg_r = (double*)take(nn * 8);
    t->cg_p0 = (double*)take(nn * 8);
    t->cg_p1 = (double*)take(nn * 8);
    t->cg_q = (double*)take(nn * 8);
    t->phi_prev = (double*)take(nn * 8);
    t->partials = (double*)take(parts * 8);
    t->mg = take(mg_bytes(cfg));
    if (cfg->same_species & 4) {
        t->rec_list = (uint32_t*)take(std::max<int64_t>(cap[1], 1) * 4);
        t->rec_v = (double*)take(std::max<int64_t>(cap[1], 1) * 24);
        t->rec_bm = (uint32_t*)take(words * 4);
        t->rec_pf = (uint32_t*)take(words * 4);
    }
    if (cfg->weighted) {
        t->fi_cnt = (uint32_t*)take(cap[2] * 4);
        t->prod_c = (uint32_t*)take(cap[2] * 4);
        for (int s = 0; s < 3; ++s) {
            t->split_list[s] = (uint32_t*)take(cap[s] * 4);
            t->split_c[s] = (uint32_t*)take(cap[s] * 4);
            t->split_v[s] = (double*)take(cap[s] * 24);
            t->split_bm[s] = (uint32_t*)take(words * 4);
            t->split_pf[s] = (uint32_t*)take(words * 4);
        }
    }
    if (c) {
        c->scan_blocks_n = scan_blocks;
        c->partials_n = parts;
        c->tmp_cap = capmax;
        c->ev_cap = cap[2];
        c->id_cap = idc;
        c->bm_words = words;
    }
    return off + 256;
}

extern "C" {

pic_status pic_scratch_size(const pic_config* cfg, const int64_t cap[3], size_t* bytes) {
    if (const char* e = check_config(cfg)) {
        (void)e;
        return PIC_E_INVALID_ARG;
    }
    if (!cap || !bytes) return PIC_E_INVALID_ARG;
    for (int s = 0; s < 3; ++s)
        if (cap[s] < 0 || cap[s] >= ((int64_t)1 << 30)) return PIC_E_INVALID_ARG;
    *bytes = scratch_layout(nullptr, cfg, cap, nullptr);
    return PIC_OK;
}

static thread_local std::string g_init_error;

pic_status pic_init(const pic_config* cfg, const pic_buffers* bufs, void* hip_stream, pic_ctx** out) {
    if (!out) return PIC_E_INVALID_ARG;
    *out = nullptr;
    if (const char* e = check_config(cfg)) {
        g_init_error = e;
        return PIC_E_INVALID_ARG;
    }
    if (!bufs) return PIC_E_INVALID_ARG;
    for (int s = 0; s < 3; ++s) {
        if (bufs->cap[s] < 0 || bufs->cap[s] >= ((int64_t)1 << 30)) return PIC_E_INVALID_ARG;
        if (bufs->cap[s] > 0 && (!bufs->x[s] || !bufs->y[s] || !bufs->z[s] || !bufs->vx[s] || !bufs->vy[s] ||
                                 !bufs->vz[s] || !bufs->id[s]))
            return PIC_E_INVALID_ARG;
    }
    if (!bufs->phi || !bufs->phi1 || !bufs->rho || !bufs->field || !bufs->field0 || !bufs->node_type || !bufs->scratch)
        return PIC_E_INVALID_ARG;
    if (((uintptr_t)bufs->scratch) % 256 != 0) return PIC_E_INVALID_ARG;
    if (cfg->weighted)
        for (int s = 0; s < 3; ++s)
            if (bufs->cap[s] > 0 && !bufs->w[s]) {
                g_init_error = "a weighted run needs the weight arrays";
                return PIC_E_INVALID_ARG;
            }
    size_t need = scratch_layout(nullptr, cfg, bufs->cap, nullptr);
    if (bufs->scratch_bytes < need) {
        g_init_error = "scratch too small";
        return PIC_E_INVALID_ARG;
    }
    pic_ctx* c = new (std::nothrow) pic_ctx();
    if (!c) return PIC_E_INVALID_ARG;
    c->cfg = *cfg;
    c->cfg.xs_el = c->cfg.xs_iz = c->cfg.xs_cx = nullptr;
    c->buf = *bufs;
    c->stream = (hipStream_t)hip_stream;
    scratch_layout(c, cfg, bufs->cap, (char*)bufs->scratch);
    Grid& g = c->g;
    g.nx = cfg->nx;
    g.ny = cfg->ny;
    g.nz = cfg->nz;
    g.h = cfg->h;
    g.R = cfg->tip_r / cfg->h;
    g.H = cfg->tip_h / cfg->h;
    g.zc = g.H - g.R;
    g.xc = 0.5 * (double)(cfg->nx - 1);
    g.yc = 0.5 * (double)(cfg->ny - 1);
    g.nn = (int64_t)cfg->nx * cfg->ny * cfg->nz;
    g.nc = (int64_t)(cfg->nx - 1) * (cfg->ny - 1) * (cfg->nz - 1);
    g.ntx = (cfg->nx - 2) / kTile + 1;
    g.nty = (cfg->ny - 2) / kTile + 1;
    g.ntz = (cfg->nz - 2) / kTile + 1;
    g.nkeys = (int64_t)g.ntx * g.nty * g.ntz * kTileCells;
    const double qm[3] = {-kQe / kMe, kQe / cfg->m_ion, 0.0};
    for (int s = 0; s < 3; ++s) c->kq[s] = qm[s] * cfg->dt * cfg->dt / cfg->h;
    // ADK constants of Eq. dfi (z = 1) and the field below which P dt < 2^-64
    c->adk_n = 3.69 / std::sqrt(cfg->xi);
    c->adk_c = 1.52 * std::pow(4.0, c->adk_n) * cfg->xi / (c->adk_n * std::tgamma(2.0 * c->adk_n));
    c->ebsi = 1.5 * std::pow(cfg->xi, 1.5);
    {
        double x32 = std::pow(cfg->xi, 1.5), e = 2.0 * c->adk_n - 1.0, dtfs = cfg->dt * 1e15;
        double lo = 1e-6, hi = c->ebsi;
        if (adk_rate(c->adk_c, e, x32, hi) * dtfs < 0x1p-64) {
            c->fi_thr = hi;
        } else {
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + hi);
                if (adk_rate(c->adk_c, e, x32, mid) * dtfs < 0x1p-64) lo = mid;
                else hi = mid;
            }
            c->fi_thr = lo;
        }
    }
    // Bounds of the collision rate u sigma_tot(E(u)) for the null-collision
    // test, per pair class (0: e-Cu, el + iz; 1: Cu+-Cu, cx): entry k bounds
    // every relative speed whose energy E = m u^2 / 2 is at most that of
    // table node k + 1. The tables are linear in ln E between nodes and u
    // grows with E, so on a segment u sigma is at most the segment's top
    // speed times the larger of its two node values; below the first node
    // sigma is the first value.
    {
        const int n = cfg->xs_n;
        const double lnr = std::log(cfg->xs_emax / cfg->xs_emin);
        c->nu_tab.assign(2 * (size_t)n, 0.0);
        for (int cls = 0; cls < 2; ++cls) {
            const double m = cls == 0 ? kMe : cfg->m_ion;
            auto sig = [&](int k) { return cls == 0 ? cfg->xs_el[k] + cfg->xs_iz[k] : cfg->xs_cx[k]; };
            auto speed = [&](int k) {
                return std::sqrt(2.0 * cfg->xs_emin * std::exp(lnr * k / (n - 1)) * kQe / m);
            };
            double cum = speed(0) * sig(0);
            for (int k = 0; k < n - 1; ++k) {
                cum = std::max(cum, speed(k + 1) * std::max(sig(k), sig(k + 1)));
                c->nu_tab[(size_t)cls * n + k] = cum;
            }
            c->nu_tab[(size_t)cls * n + n - 1] = cum;
        }
    }
    c->npatch = fn_patches(cfg);
    c->evap_flux = evaporation_flux(cfg->m_ion, cfg->surface_T);
    c->evap_vsig = std::sqrt(1.380649e-23 * cfg->surface_T / cfg->m_ion) * cfg->dt / cfg->h;

    pic_status st = PIC_OK;
    auto H = [&](hipError_t e, const char* w) {
        if (st == PIC_OK) st = hip_check(c, e, w);
    };
    H(hipHostMalloc((void**)&c->host_st, sizeof(DevState) + 256, hipHostMallocDefault), "hipHostMalloc");
    if (st != PIC_OK) {
        g_init_error = c->err;
        delete c;
        return st;
    }
    hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1), 0, c->stream, c->st);
    H(hipMemcpyAsync(c->xs, cfg->xs_el, cfg->xs_n * 8, hipMemcpyHostToDevice, c->stream), "copy tables");
    H(hipMemcpyAsync(c->xs + cfg->xs_n, cfg->xs_iz, cfg->xs_n * 8, hipMemcpyHostToDevice, c->stream), "copy tables");
    H(hipMemcpyAsync(c->xs + 2 * cfg->xs_n, cfg->xs_cx, cfg->xs_n * 8, hipMemcpyHostToDevice, c->stream),
      "copy tables");
    H(hipMemcpyAsync(c->xs + 3 * cfg->xs_n, c->nu_tab.data(), 2 * cfg->xs_n * 8, hipMemcpyHostToDevice, c->stream),
      "copy tables");
    uint32_t* ids[3] = {bufs->id[0], bufs->id[1], bufs->id[2]};
    H(hipMemcpyAsync(c->id_ptrs, ids, sizeof(ids), hipMemcpyHostToDevice, c->stream), "copy id pointers");
    H(launch_zero(c->dyn, 64 * 4, c->stream), "zero");
    H(launch_zero(c->nflag, bufs->cap[2] * 4, c->stream), "zero");
    for (int k = 0; k < 2; ++k) H(launch_zero(c->bitmap[k], c->bm_words * 4, c->stream), "zero");
    H(launch_zero(c->off, ((size_t)g.nkeys + 1) * 4, c->stream), "zero");
    if (cfg->weighted)
        for (int k = 0; k < 3; ++k) H(launch_zero(c->split_bm[k], c->bm_words * 4, c->stream), "zero");
    if (c->rec_bm) H(launch_zero(c->rec_bm, c->bm_words * 4, c->stream), "zero");
    H(launch_zero(bufs->rho, g.nn * 8, c->stream), "zero");
    H(static_work_setup(&c->static_work), "static work array");
    H(launch_node_types(c), "node types");
    if (st == PIC_OK) {
        int r = mg_setup(c);
        if (r == -2) st = fail(c, PIC_E_HIP, "multigrid setup failed");
    }
    // unit-anode Laplace problem: phi1, its field (Shockley-Ramo weighting
    // field) and the anode voltage that gives the requested apex field
    pic_solve_info info{};
    if (st == PIC_OK) {
        int r = cg_solve(c, bufs->phi1, 1.0, bufs->rho, PIC_GUESS_ZERO, cfg->laplace_rtol, 1000000, &info);
        if (r != 0) st = fail(c, PIC_E_HIP, "Laplace solve failed");
        else if (!info.converged) st = fail(c, PIC_E_NOT_CONVERGED, "Laplace solve did not converge");
    }
    if (st == PIC_OK) {
        H(apex_interp(c, bufs->phi1, g.xc, g.yc, g.H + 1.0, c->mom_out), "apex");
        double v = 0.0;
        H(hipMemcpyAsync(&v, c->mom_out, 8, hipMemcpyDeviceToHost, c->stream), "apex copy");
        H(hipStreamSynchronize(c->stream), "sync");
        c->F1 = v / cfg->h;
        if (!(c->F1 > 0)) st = fail(c, PIC_E_INVALID_ARG, "non-positive Laplace apex field");
        else c->V0 = cfg->apex_field / c->F1;
    }
    if (st == PIC_OK) {
        H(launch_field(c, bufs->phi1, bufs->field0), "field0");
        int64_t G = (g.nn + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(k_scale, dim3((unsigned)G), dim3(kBlock), 0, c->stream, bufs->phi, bufs->phi1, c->V0, g.nn);
        H(launch_field(c, bufs->phi, bufs->field), "field");
        // the gap voltage starts at the applied voltage; from now on, with
        // the circuit, the solves hold the anode at it (after the unit-anode
        // Laplace solve above, which must not)
        hipLaunchKernelGGL(k_set_vgap, dim3(1), dim3(1), 0, c->stream, c->st, c->V0);
        c->circuit = cfg->circuit_R > 0.0;
        H(hipStreamSynchronize(c->stream), "sync");
    }
    if (st != PIC_OK) {
        g_init_error = c->err;
        (void)hipHostFree(c->host_st);
        mg_free(c);
        delete c;
        return st;
    }
    c->last_solve = info;
    *out = c;
    return PIC_OK;
}

static pic_status sync_state(pic_ctx* c) {
    pic_status s = hip_check(c, hipMemcpyAsync(c->host_st, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream),
                             "state copy");
    if (s != PIC_OK) return s;
    s = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    if (s != PIC_OK) return s;
    if (c->host_st->error != 0) {
        int e = c->host_st->error;
        return fail(c, e, e == PIC_E_CAPACITY   ? "particle capacity exceeded (or a cell holds more than 4096 particles)"
                          : e == PIC_E_OVERFLOW ? "possible fixed-point charge overflow: a tile of 8^3 cells holds 2^20 "
                                                  "or more particles"
                                                : "device error");
    }
    return PIC_OK;
}

pic_status pic_inject(pic_ctx* c, const pic_particles* src, int64_t* n_added) {
    if (!c) return PIC_E_INVALID_ARG;
    if (c->failed) return PIC_E_STATE;
    if (n_added) *n_added = 0;
    pic_status s = sync_state(c);
    if (s != PIC_OK) return s;
    if (src) {
        if (src->species < 0 || src->species > 2 || src->n < 0) return fail(c, PIC_E_INVALID_ARG, "bad particle load");
        if (src->n > 0 && (!src->x || !src->y || !src->z || !src->vx || !src->vy || !src->vz))
            return fail(c, PIC_E_INVALID_ARG, "NULL particle array");
        if ((int64_t)c->host_st->n_slots[src->species] + src->n > c->buf.cap[src->species])
            return fail(c, PIC_E_CAPACITY, "particle capacity exceeded by the load");
        s = hip_check(c, load_particles(c, src), "load");
        if (s != PIC_OK) return s;
        s = sync_state(c);
        if (s == PIC_OK && n_added) *n_added = src->n;
        c->bins_valid = 0;
        c->need_sort = 1;  // order the load by cell at the next collide phase
        c->phi_hist = 0;
        return s;
    }
    unsigned long long before = c->host_st->injected;
    s = hip_check(c, inject_phase(c), "inject");
    if (s != PIC_OK) return s;
    s = sync_state(c);
    if (s == PIC_OK && n_added) *n_added = (int64_t)(c->host_st->injected - before);
    c->bins_valid = 0;
    return s;
}

pic_status pic_inject_noalloc(pic_ctx* c, int64_t* n_added) {
    if (!c) return PIC_E_INVALID_ARG;
    if (c->failed) return PIC_E_STATE;
    if (n_added) *n_added = 0;
    const size_t need = inject_work_bytes(c->npatch);
    if (need > kStaticWorkBytes)
        return fail(c, PIC_E_INVALID_ARG,
                    "emission of " + std::to_string(c->npatch) + " patches needs " + std::to_string(need) +
                        " bytes of work memory, more than the " + std::to_string(kStaticWorkBytes) +
                        "-byte static array of pic_inject_noalloc");
    if (!c->static_work) return fail(c, PIC_E_STATE, "static work array not set up");
    pic_status s = sync_state(c);
    if (s != PIC_OK) return s;
    unsigned long long before = c->host_st->injected;
    uint32_t* cnt = (uint32_t*)c->static_work;
    double* part = (double*)((char*)c->static_work + (((size_t)c->npatch * 4 + 255) & ~(size_t)255));
    s = hip_check(c, inject_phase_in(c, cnt, part), "inject");
    if (s != PIC_OK) return s;
    s = sync_state(c);
    if (s == PIC_OK && n_added) *n_added = (int64_t)(c->host_st->injected - before);
    c->bins_valid = 0;
    return s;
}

static pic_status solve(pic_ctx* c, int solver, int guess, double rtol, int maxit, pic_solve_info* info) {
    pic_solve_info tmp{};
    if (!info) info = &tmp;
    int th = tic(c, PIC_T_SOLVE);
    int r;
    int fell_back = 0;
    if (guess == PIC_GUESS_LEARNED && !c->learn_fallback) {
        r = guess_phi(c, true);
        if (r != 0) return fail(c, PIC_E_HIP, "warm start failed");
        guess = PIC_GUESS_PREVIOUS;
    } else if (guess == PIC_GUESS_LEARNED) {
        // The network's guess is judged against V0 phi1 by the initial
        // residual of each (a zero-iteration CG pass: the residual and its
        // norm only); a guess that is not finite, or worse, is replaced.
        pic_solve_info i_plain{}, i_net{};
        r = guess_phi(c, false);
        if (r == 0) r = cg_solve(c, c->buf.phi, c->V0, c->buf.rho, PIC_GUESS_PREVIOUS, rtol, 0, &i_plain);
        if (r == 0) r = guess_phi(c, true);
        if (r == 0) r = cg_solve(c, c->buf.phi, c->V0, c->buf.rho, PIC_GUESS_PREVIOUS, rtol, 0, &i_net);
        if (r != 0) return fail(c, PIC_E_HIP, "warm start failed");
        fell_back = c->host_st->learn_bad || !std::isfinite(i_net.relres0) || !(i_net.relres0 <= i_plain.relres0);
        if (fell_back) {
            r = guess_phi(c, false);
            if (r != 0) return fail(c, PIC_E_HIP, "warm start failed");
        }
        guess = PIC_GUESS_PREVIOUS;
    } else if (guess == PIC_GUESS_LAPLACE) {
        r = guess_phi(c, false);
        if (r != 0) return fail(c, PIC_E_HIP, "warm start failed");
        guess = PIC_GUESS_PREVIOUS;
    }
    if (solver == PIC_SOLVER_CG)
        r = cg_solve(c, c->buf.phi, c->V0, c->buf.rho, guess, rtol, maxit, info);
    else if (solver == PIC_SOLVER_MGCG)
        r = mgcg_solve(c, c->buf.phi, c->V0, c->buf.rho, guess, rtol, maxit, info);
    else
        r = mixed_solve(c, c->buf.phi, c->V0, c->buf.rho, guess, rtol, maxit, info);
    if (r == -3) return fail(c, PIC_E_INVALID_ARG, "solver not available for this configuration");
    if (r != 0) return fail(c, PIC_E_HIP, "solver failed");
    info->fell_back = fell_back;
    c->last_solve = *info;
    c->cg_iters_total += info->iterations;
    pic_status s = hip_check(c, launch_field(c, c->buf.phi, c->buf.field), "field");
    toc(c, th);
    if (s != PIC_OK) return s;
    if (!info->converged) return fail(c, PIC_E_NOT_CONVERGED, "Poisson solve did not converge");
    return PIC_OK;
}

// The side stream (default priority) and its two events, created on first use.
static hipError_t side_init(pic_ctx* c) {
    if (c->side_stream) return hipSuccess;
    hipError_t e = hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_dep, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_col, hipEventDisableTiming);
    return e;
}

pic_status pic_step(pic_ctx* c, int32_t nsteps, uint32_t flags) {
    if (!c) return PIC_E_INVALID_ARG;
    if (c->failed) return PIC_E_STATE;
    if (nsteps < 0) return fail(c, PIC_E_INVALID_ARG, "nsteps < 0");
    pic_status result = PIC_OK;
    for (int32_t n = 0; n < nsteps; ++n) {
        pic_status s = PIC_OK;
        if (c->prof && c->ev_n > c->ev_max / 4) flush_timers(c);
        int th = tic(c, PIC_T_STEP);
        if (flags & PIC_STEP_INJECT) {
            int t = tic(c, PIC_T_INJECT);
            s = hip_check(c, inject_phase(c), "inject");
            toc(c, t);
        }
        if (s == PIC_OK && (flags & (PIC_STEP_PUSH | PIC_STEP_DEPOSIT))) {
            int t = tic(c, PIC_T_PARTICLES);
            s = hip_check(c, particles_phase(c, (flags & PIC_STEP_PUSH) != 0), "push");
            toc(c, t);
        }
        // The collisions touch only the particles and their bins, the solve
        // only the charge (already deposited), the potential and the field,
        // so without profiling a step that does both runs its collisions on
        // the side stream, concurrently with the solve.
        // A step that merges superparticles, or recombines, corrects the
        // charge after its collisions, so its solve waits for them.
        const bool side = !c->prof && (flags & PIC_STEP_COLLIDE) && (flags & PIC_STEP_SOLVE) && !merge_step(c) &&
                          !(c->cfg.same_species & 4);
        bool joined = true;
        if (s == PIC_OK && (flags & PIC_STEP_COLLIDE)) {
            if (!c->bins_valid) return fail(c, PIC_E_INVALID_ARG, "the collide phase needs a push or deposit phase first");
            if (side) {
                s = hip_check(c, side_init(c), "side stream");
                if (s != PIC_OK) return s;
                s = hip_check(c, hipEventRecord(c->ev_dep, c->stream), "event");
                if (s == PIC_OK) s = hip_check(c, hipStreamWaitEvent(c->side_stream, c->ev_dep, 0), "event");
                if (s != PIC_OK) return s;
                hipStream_t keep = c->stream;
                c->stream = c->side_stream;
                hipError_t e = collide_phase(c, (flags & PIC_STEP_EVENTS) != 0);
                if (e == hipSuccess) e = hipEventRecord(c->ev_col, c->side_stream);
                c->stream = keep;
                s = hip_check(c, e, "collide");
                joined = false;
            } else {
                int t = tic(c, PIC_T_COLLIDE);
                s = hip_check(c, collide_phase(c, (flags & PIC_STEP_EVENTS) != 0), "collide");
                toc(c, t);
            }
        }
        if (s == PIC_OK && (flags & PIC_STEP_SOLVE)) {
            // guess: the previous potential, or phi_n + (phi_n - phi_{n-1})
            // once two step solves are on record (phi_prev keeps phi_n)
            if (c->cfg.step_guess == 1) s = hip_check(c, extrapolate_phi(c, c->phi_hist >= 2), "extrapolation");
            if (s == PIC_OK)
                s = solve(c, c->cfg.solver, PIC_GUESS_PREVIOUS, c->cfg.step_rtol, c->cfg.step_maxit, nullptr);
            if (s == PIC_E_NOT_CONVERGED) {
                result = s;
                s = PIC_OK;
                c->phi_hist = 0;
            } else if (s == PIC_OK) {
                c->phi_hist = c->phi_hist < 2 ? c->phi_hist + 1 : 2;
            }
        } else if (s == PIC_OK && (flags & PIC_STEP_FIELD)) {
            s = hip_check(c, launch_field(c, c->buf.phi, c->buf.field), "field");
        }
        // everything after this step on the library stream follows its collisions
        if (!joined) {
            pic_status sj = hip_check(c, hipStreamWaitEvent(c->stream, c->ev_col, 0), "event");
            if (s == PIC_OK) s = sj;
        }
        toc(c, th);
        if (s != PIC_OK) return s;
        if (flags & PIC_STEP_ADVANCE) c->step++;
    }
    return result;
}

pic_status pic_solve_poisson(pic_ctx* c, int32_t solver, int32_t guess, double rtol, int32_t maxit,
                             pic_solve_info* info) {
    if (!c) return PIC_E_INVALID_ARG;
    if (c->failed) return PIC_E_STATE;
    if (solver < PIC_SOLVER_CG || solver > PIC_SOLVER_MIXED || guess < PIC_GUESS_ZERO || guess > PIC_GUESS_LEARNED ||
        (guess == PIC_GUESS_LEARNED && !c->learned) ||
        !(rtol > 0) || maxit < 0)
        return fail(c, PIC_E_INVALID_ARG, "bad solver arguments");
    if (c->prof && c->ev_n > c->ev_max / 4) flush_timers(c);
    c->phi_hist = 0;  // the potential no longer follows the step sequence
    return solve(c, solver, guess, rtol, maxit, info);
}

pic_status pic_moments(pic_ctx* c, pic_moments_t* out) {
    if (!c || !out) return PIC_E_INVALID_ARG;
    if (c->failed) return PIC_E_STATE;
    pic_status s = hip_check(c, moments_phase(c, c->mom_out), "moments");
    if (s != PIC_OK) return s;
    double host[11];
    s = hip_check(c, hipMemcpyAsync(host, c->mom_out, sizeof(host), hipMemcpyDeviceToHost, c->stream), "copy");
    if (s != PIC_OK) return s;
    s = sync_state(c);
    std::memset(out, 0, sizeof(*out));
    const DevState* h = c->host_st;
    for (int k = 0; k < 3; ++k) {
        out->n_alive[k] = (int64_t)llround(host[k]);
        out->n_slots[k] = (int64_t)h->n_slots[k];
        out->ke[k] = host[3 + k];
        for (int b = 0; b < 5; ++b) out->absorbed[k][b] = (int64_t)h->absorbed[k][b];
    }
    for (int k = 0; k < 5; ++k) out->events[k] = (int64_t)h->events[k];
    out->injected = (int64_t)h->injected;
    out->fn_clamped = (int64_t)h->fn_clamped;
    out->bsi_count = (int64_t)h->bsi_count;
    long long q;
    std::memcpy(&q, &host[7], 8);
    out->q_total = q;
    out->next_id = (int64_t)h->next_id;
    out->step = c->step;
    out->i_sr = host[6];
    out->fn_expected = h->fn_expected;
    out->v0 = c->V0;
    out->apex_field1 = c->F1;
    out->error = h->error;
    out->last_cg_iters = c->last_solve.iterations;
    out->last_cg_relres = c->last_solve.relres;
    out->cg_iters_total = c->cg_iters_total;
    out->evaporated = (int64_t)h->evaporated;
    out->evap_expected = h->evap_expected;
    out->bomb_energy[0] = h->bomb_e[0];
    out->bomb_energy[1] = h->bomb_e[1];
    out->v_gap = h->v_gap;
    out->i_gap = h->i_gap;
    out->i_tot = h->i_tot;
    for (int k = 0; k < 3; ++k) out->n_phys[k] = (int64_t)llround(host[8 + k]);
    for (int k = 0; k < 5; ++k) out->events_w[k] = (int64_t)h->events_w[k];
    out->splits = (int64_t)h->splits;
    out->evap_atoms = (int64_t)h->evap_atoms;
    for (int s = 0; s < 3; ++s) out->merges[s] = (int64_t)h->merges[s];
    out->nn_events = (int64_t)h->nn_events;
    out->coulomb_pairs = (int64_t)h->coulomb_pairs;
    out->recombinations = (int64_t)h->recombinations;
    return s;
}

pic_status pic_events(pic_ctx* c, pic_event* out, int64_t cap, int64_t* n) {
    if (!c || !n || cap < 0 || (cap > 0 && !out)) return PIC_E_INVALID_ARG;
    if (c->failed) return PIC_E_STATE;
    pic_status s = sync_state(c);
    if (s != PIC_OK) return s;
    int64_t have = std::min<int64_t>((int64_t)c->host_st->n_ev, c->ev_cap);
    *n = have;
    int64_t m = std::min(have, cap);
    if (m > 0) {
        s = hip_check(c, hipMemcpyAsync(out, c->ev, m * sizeof(pic_event), hipMemcpyDeviceToHost, c->stream), "copy");
        if (s == PIC_OK) s = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    }
    return s;
}

const char* pic_last_error(const pic_ctx* c) {
    if (!c) return g_init_error.c_str();
    return c->err.c_str();
}

void pic_destroy(pic_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    if (c->evpool) {
        for (int i = 0; i < c->ev_max; ++i) (void)hipEventDestroy(c->evpool[i]);
        delete[] c->evpool;
        delete[] c->ev_slot;
    }
    if (c->host_st) (void)hipHostFree(c->host_st);
    if (c->pcg_exec) (void)hipGraphExecDestroy(c->pcg_exec);
    if (c->pcg_graph) (void)hipGraphDestroy(c->pcg_graph);
    if (c->mix_exec) (void)hipGraphExecDestroy(c->mix_exec);
    if (c->mix_graph) (void)hipGraphDestroy(c->mix_graph);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->side_stream) {
        (void)hipStreamSynchronize(c->side_stream);
        (void)hipStreamDestroy(c->side_stream);
    }
    if (c->ev_dep) (void)hipEventDestroy(c->ev_dep);
    if (c->ev_col) (void)hipEventDestroy(c->ev_col);
    mg_free(c);
    delete c;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Profiling timers

namespace pic {

void flush_timers(pic_ctx* c) {
    if (!c->evpool || c->ev_n == 0) return;
    (void)hipStreamSynchronize(c->stream);
    for (int i = 0; i + 1 < c->ev_n; i += 2) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->evpool[i], c->evpool[i + 1]) == hipSuccess) {
            int s = c->ev_slot[i / 2];
            c->t_ms[s] += ms;
            c->t_cnt[s] += 1;
        }
    }
    c->ev_n = 0;
}

// Handles stay valid until the next flush, which happens only at the start of
// an entry point (no interval is open then); a full pool skips timing.
int tic(pic_ctx* c, int slot) {
    if (!c->prof || c->ev_n + 2 > c->ev_max) return -1;
    int h = c->ev_n;
    c->ev_n += 2;
    c->ev_slot[h / 2] = slot;
    (void)hipEventRecord(c->evpool[h], c->stream);
    return h;
}

void toc(pic_ctx* c, int h) {
    if (h < 0 || !c->prof) return;
    (void)hipEventRecord(c->evpool[h + 1], c->stream);
}

}  // namespace pic

extern "C" {

pic_status pic_profile(pic_ctx* c, int32_t enable) {
    if (!c) return PIC_E_INVALID_ARG;
    if (enable && !c->evpool) {
        c->ev_max = 16384;
        c->evpool = new hipEvent_t[c->ev_max];
        c->ev_slot = new int[c->ev_max / 2];
        for (int i = 0; i < c->ev_max; ++i)
            if (hipEventCreate(&c->evpool[i]) != hipSuccess) return PIC_E_HIP;
    }
    if (!enable) flush_timers(c);
    c->prof = enable ? 1 : 0;
    return PIC_OK;
}

pic_status pic_timers(pic_ctx* c, double* ms, int64_t* count, int32_t reset) {
    if (!c) return PIC_E_INVALID_ARG;
    flush_timers(c);
    for (int i = 0; i < PIC_NTIMERS; ++i) {
        if (ms) ms[i] = c->t_ms[i];
        if (count) count[i] = c->t_cnt[i];
        if (reset) {
            c->t_ms[i] = 0.0;
            c->t_cnt[i] = 0;
        }
    }
    return PIC_OK;
}

}  // extern "C"
