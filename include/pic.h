/*
 * pic.h -- C interface of libpic, an MI355X (gfx950) implementation of the
 * electrostatic particle-in-cell step with Monte Carlo collisions of
 * "Simulating vacuum arc initiation by coupling emission, heating and plasma
 * processes" (arXiv 2402.08404, Sec. 2.1-2.3).
 *
 * One context holds one instance: a 3D node grid with a grounded cathode plane
 * carrying a Cu nanotip (cylinder + hemispherical cap, held at 0 V), an anode
 * plane at V0 and lateral faces with zero normal field (Sec. 2.1, bcf1-bcf3);
 * three species (electrons, Cu+ ions, Cu neutrals); field emission from the
 * tip; and a Poisson solve per step (Eq. poi).
 *
 * Units of the particle state: positions in grid units X = x/h (node (i,j,k)
 * at X=i), velocities in grid units per step V = v dt / h. Node fields are
 * stored as 4 values per node (Ex, Ey, Ez, 0) in V/m. Charge density is an
 * int64 per node in units of 2^-40 e.
 *
 * Memory: every device buffer (particles, grids, scratch) is allocated and
 * owned by the caller and must outlive the context; the library never frees
 * them. Host pointers in pic_config are read during pic_init only.
 *
 * Threading: a context is bound to one HIP stream and is not thread-safe.
 * All calls enqueue work on that stream; calls that return host data
 * (pic_moments, pic_events, pic_solve_poisson, pic_inject) synchronize it.
 *
 * Errors: every call returns PIC_OK (0) or a negative pic_status. Device-side
 * conditions (particle capacity; a possible fixed-point overflow of the
 * charge, reported when a tile of 8^3 cells holds 2^20 or more particles, the
 * count below which no node sum can reach 2^63; a cell with more particles
 * than the collision kernels accept) are sticky: they are raised by the next
 * synchronizing call and leave the context in a failed state in which every
 * call returns PIC_E_STATE. pic_last_error gives a message.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pic_status;
#define PIC_OK 0
#define PIC_E_INVALID_ARG (-1)
#define PIC_E_HIP (-2)
#define PIC_E_CAPACITY (-3)
#define PIC_E_OVERFLOW (-4)
#define PIC_E_NOT_CONVERGED (-5)
#define PIC_E_STATE (-6)

/* precision of the particle state and of the node field */
#define PIC_F64 0
#define PIC_F32 1

/* Poisson solver */
#define PIC_SOLVER_CG 0      /* plain FP64 conjugate gradients */
#define PIC_SOLVER_MGCG 1    /* FP64 CG preconditioned by a multigrid V-cycle */
#define PIC_SOLVER_MIXED 2   /* FP32 inner CG with FP64 dots, FP64 residual refinement */

/* species */
#define PIC_ELECTRON 0
#define PIC_ION 1
#define PIC_NEUTRAL 2

/* initial guess of pic_solve_poisson */
#define PIC_GUESS_ZERO 0
#define PIC_GUESS_PREVIOUS 1
#define PIC_GUESS_LAPLACE 2   /* V0 phi1: the exact charge-free solution */
#define PIC_GUESS_LEARNED 3   /* V0 phi1 plus the network's charge response (pic_set_learned_guess) */

/* phases of pic_step; each step runs the selected phases in this order */
#define PIC_STEP_INJECT 0x01   /* Fowler-Nordheim emission from the tip, then the evaporation of neutrals
                                  when cfg.surface_T > 0 (Sec. 2.3.1) */
#define PIC_STEP_PUSH 0x02     /* gather, leapfrog push, boundary removal, deposit, binning (Sec. 2.2);
                                  the bombardment energy of ions reaching the cathode (Sec. 2.3.3); with the
                                  circuit, the Shockley-Ramo current of the push and one step of the RC
                                  circuit, whose gap voltage is the anode potential of the next solves */
#define PIC_STEP_DEPOSIT 0x04  /* deposit and binning at the current positions, no motion */
#define PIC_STEP_COLLIDE 0x08  /* MCC (Eqs. colp, du, newv), field ionization (Eq. dfi), products */
#define PIC_STEP_SOLVE 0x10    /* Poisson solve (Eq. poi) from the previous potential (or its extrapolation, cfg.step_guess), then the field */
#define PIC_STEP_FIELD 0x20    /* node field from the current potential only */
#define PIC_STEP_ADVANCE 0x40  /* advance the step counter */
#define PIC_STEP_EVENTS 0x80   /* record the collision events of this step (pic_events) */
#define PIC_STEP_FULL (PIC_STEP_INJECT | PIC_STEP_PUSH | PIC_STEP_COLLIDE | PIC_STEP_SOLVE | PIC_STEP_ADVANCE)

/* event kinds */
#define PIC_EV_ELASTIC 1   /* e + Cu -> e + Cu */
#define PIC_EV_IONIZE 2    /* e + Cu -> Cu+ + 2e */
#define PIC_EV_CX 3        /* Cu+ + Cu -> Cu + Cu+ */
#define PIC_EV_FIELD_ION 4 /* Cu -> Cu+ + e in the local field */

typedef struct pic_config {
    int32_t nx, ny, nz;    /* nodes per axis, each >= 4 */
    int32_t precision;     /* PIC_F64 or PIC_F32 */
    double h;              /* node spacing [m] */
    double tip_r;          /* tip radius [m] */
    double tip_h;          /* total tip height to the apex [m], >= tip_r */
    double apex_field;     /* requested Laplace field just above the apex [V/m] */
    double phi_w;          /* work function [eV] */
    double dt;             /* time step [s] */
    double xi;             /* first ionization energy of Cu [eV] */
    double m_ion;          /* Cu mass [kg] */
    uint64_t seed;         /* Philox4x32-10 key */
    int32_t xs_n;          /* cross-section table length, >= 2 */
    int32_t solver;        /* PIC_SOLVER_* used by PIC_STEP_SOLVE */
    double xs_emin, xs_emax;              /* energies of the first and last table node [eV] */
    const double* xs_el;                  /* host: e-Cu elastic cross section [m^2] */
    const double* xs_iz;                  /* host: e-Cu impact ionization [m^2] */
    const double* xs_cx;                  /* host: Cu+-Cu charge exchange [m^2] */
    int32_t fn_rings;      /* emission patches: rings on the cap */
    int32_t fn_az;         /* emission patches: azimuths per ring */
    double laplace_rtol;   /* tolerance of the unit-anode Laplace solve at init (e.g. 1e-13) */
    double step_rtol;      /* tolerance of the solve inside pic_step (e.g. 1e-8) */
    int32_t step_maxit;    /* iteration limit of the solve inside pic_step */
    int32_t sort_every;    /* reorder particles by cell every this many collide phases (0: never) */
    int64_t id_capacity;   /* largest particle id + 1 the run may reach (0: 8 x total capacity) */
    int32_t stencil_blocks; /* about this many blocks per z-marching solver kernel (0: 1024; 64..4096) */
    int32_t step_guess;    /* guess of the solve inside pic_step: 0 the previous potential, 1 linear
                              extrapolation 2 phi_n - phi_{n-1} from the two previous step solves */
    /* Surface and circuit terms (Sec. 2.3.1): */
    double surface_T;      /* prescribed uniform tip surface temperature [K] for the Clausius-Clapeyron
                              evaporation of neutrals in the inject phase (0: no evaporation) */
    double circuit_R;      /* series resistance [ohm] of the RC circuit (0: the anode stays at V0) */
    double circuit_C;      /* gap capacitance [F] of the RC circuit */
    /* Superparticle weights (Sec. 2.3.2): */
    int32_t weighted;      /* 1: every superparticle carries an integer weight (pic_buffers.w; physical
                              particles per superparticle, the smallest weight w_min being 1); collisions
                              split superparticles; 0: every weight is 1 and no weight array is read */
    int32_t w_max;         /* largest weight that the injection rule gives evaporated neutrals and that
                              merging creates (<= 1: injection weights 1, no merging) */
    double n_max;          /* superparticle density [1/m^3] of the injection rule (1e24 = 1e-6 per A^3) */
    /* Merging of superparticles (Sec. 2.3.2; needs weighted = 1): in the collide phase of every step
     * whose counter is a multiple of merge_every, per cell and species, the superparticles binned by
     * the push that are still alive are taken in ascending id order; when there are N > merge_max of
     * them, the first min(floor(N/2), N - merge_max) consecutive pairs merge into one superparticle of
     * weight w1 + w2 at the weighted mean position and velocity (the centre of mass), keeping the lower
     * id; a pair whose summed weight would exceed w_max is left alone. The node charge is corrected
     * exactly (integer deposit), and such a step runs its collisions before the solve. */
    int32_t merge_every;   /* 0: no merging */
    int32_t merge_max;     /* >= 1 when merge_every > 0 */
    /* Same-species and Coulomb pairing (Table colls: Cu + Cu elastic, Coulomb collisions of all charged
     * particles after Takizuka and Abe; needs weighted = 0): in the collide phase, after the collisions
     * and products, per cell the particles of one species binned by the push, in ascending id order
     * rotated by floor(U_c N), are paired consecutively. Cu + Cu: hard spheres of cross section
     * sigma_nn, P = 1 - exp(-u n sigma_nn dt), n = N / h^3, isotropic scattering; neutrals with an event
     * this step and, for odd N, the last one sit out. Coulomb: every pair's relative velocity turns by
     * 2 atan(delta), delta normal of variance e^4 n_L ln(Lambda) dt / (8 pi eps0^2 mu^2 u^3); odd N: the
     * first three collide pairwise with dt / 2; e-Cu+: each particle of the more numerous species meets
     * one of the other (reused cyclically), n_L the smaller density. */
    int32_t same_species;  /* bit 0: Cu + Cu elastic, bit 1: Coulomb, bit 2: recombination; 0: none */
    int32_t reserved2;
    double sigma_nn;       /* Cu-Cu elastic cross section [m^2] */
    double coulomb_log;    /* Coulomb logarithm ln(Lambda), > 0 with the Coulomb bit */
    /* Recombination Cu+ + e -> Cu (Table colls), after the Coulomb pairs: electrons and ions of a cell
     * paired like the collision classes (the fewer species, tie: the ions, as projectiles in id order,
     * targets shifted by floor(U_c N_t)); a pair recombines when U < 1 - exp(-u n sigma_rec dt),
     * n = N_t / h^3; the atom takes the ion's position, the pair's centre-of-mass velocity and a new id
     * (ascending ion ids, after the ionization products); both charges leave the node charge. A step
     * with recombination runs its collisions before the solve. */
    double sigma_rec;      /* recombination cross section [m^2] */
} pic_config;

typedef struct pic_buffers {
    /* per species s: SoA of capacity cap[s]; element type double (PIC_F64)
     * or float (PIC_F32) */
    void* x[3];
    void* y[3];
    void* z[3];
    void* vx[3];
    void* vy[3];
    void* vz[3];
    uint32_t* id[3];       /* 0xFFFFFFFF marks a free slot */
    int64_t cap[3];
    double* phi;           /* nx*ny*nz potential [V] */
    double* phi1;          /* nx*ny*nz unit-anode Laplace potential, written by pic_init */
    int64_t* rho;          /* nx*ny*nz node charge [2^-40 e] */
    void* field;           /* 4*nx*ny*nz node field [V/m], element type as the particles */
    void* field0;          /* 4*nx*ny*nz field of phi1 [1/m] (Shockley-Ramo weighting field) */
    uint8_t* node_type;    /* nx*ny*nz: 0 free, 1 held at 0 V, 2 held at V0 */
    void* scratch;         /* work memory of pic_scratch_size bytes, 256-byte aligned */
    size_t scratch_bytes;
    uint32_t* w[3];        /* with cfg.weighted: the weight of every slot per species (capacity cap[s]) */
} pic_buffers;

typedef struct pic_particles {
    int32_t species;       /* PIC_ELECTRON, PIC_ION or PIC_NEUTRAL */
    int32_t pad;
    int64_t n;
    const void *x, *y, *z, *vx, *vy, *vz;  /* device arrays of n elements, same type as the state */
    const uint32_t* w;     /* device weights of the n particles (NULL: weight 1); read with cfg.weighted */
} pic_particles;

typedef struct pic_solve_info {
    int32_t iterations;    /* CG iterations (matrix products) */
    int32_t converged;     /* 1 if ||r|| <= rtol ||b|| was reached */
    double relres;         /* final ||r|| / ||b|| (recursively updated residual) */
    double relres0;        /* ||r|| / ||b|| of the initial guess the solve started from */
    int32_t fell_back;     /* PIC_GUESS_LEARNED with the fallback on: 1 if the network's guess was not finite
                              or had a larger initial residual than V0 phi1, which the solve then started
                              from instead */
    int32_t reserved;
} pic_solve_info;

typedef struct pic_moments_t {
    int64_t n_alive[3];        /* alive particles per species */
    int64_t n_slots[3];        /* used slots (alive and free) per species */
    int64_t absorbed[3][5];    /* cumulative removals by boundary: 1 cathode, 2 anode, 3 lateral, 4 tip */
    int64_t events[5];         /* cumulative events by kind (PIC_EV_*) */
    int64_t injected;          /* cumulative emitted electrons */
    int64_t fn_clamped;        /* cumulative emission patches evaluated with f clamped at 1 */
    int64_t bsi_count;         /* cumulative neutrals seen above the barrier-suppression field */
    int64_t q_total;           /* sum of rho [2^-40 e] */
    int64_t next_id;           /* next particle id to be assigned */
    int64_t step;              /* step counter */
    double ke[3];              /* kinetic energy per species [J] */
    double i_sr;               /* Shockley-Ramo gap current of the stored state [A] */
    double fn_expected;        /* cumulative expected number of emitted electrons */
    double v0;                 /* anode potential [V] */
    double apex_field1;        /* Laplace apex field per volt of anode potential [1/m] */
    int32_t error;             /* sticky error code, PIC_OK if none */
    int32_t last_cg_iters;     /* iterations of the last Poisson solve */
    double last_cg_relres;     /* final relative residual of the last solve */
    int64_t cg_iters_total;    /* iterations of all solves since pic_init (the init solve excluded) */
    /* surface and circuit terms */
    int64_t evaporated;        /* cumulative evaporated neutrals */
    double evap_expected;      /* cumulative expected number of evaporated neutrals */
    double bomb_energy[2];     /* cumulative kinetic energy [J] of ions absorbed at the cathode plane and the tip
                                  (the bombardment energy E_b of Sec. 2.3.3; no sputtering, E_s = 0) */
    double v_gap;              /* gap voltage = anode potential [V] (V0 without the circuit) */
    double i_gap;              /* Shockley-Ramo current of the last push [A] (circuit only) */
    double i_tot;              /* circuit current (V0 - V_gap) / R of the last circuit step [A] */
    /* superparticle weights */
    int64_t n_phys[3];         /* physical particles per species (sum of the weights of the alive) */
    int64_t events_w[5];       /* cumulative physical collisions per event kind (sum of N_coll) */
    int64_t splits;            /* cumulative superparticles split off by partial collisions */
    int64_t evap_atoms;        /* cumulative evaporated atoms (the weights of the evaporated neutrals) */
    int64_t merges[3];         /* cumulative merged pairs per species */
    int64_t nn_events;         /* cumulative Cu + Cu elastic collisions */
    int64_t coulomb_pairs;     /* cumulative Coulomb scatterings (pairs with u > 0) */
    int64_t recombinations;    /* cumulative Cu+ + e -> Cu recombinations */
} pic_moments_t;

typedef struct pic_event {
    int32_t kind;              /* PIC_EV_* */
    uint32_t id_a;             /* electron (elastic, ionize) or ion (cx); 0xFFFFFFFF for field ionization */
    uint32_t id_b;             /* the neutral */
    uint32_t new_ion, new_e;   /* ids of the products (ionize, field ionization), else 0xFFFFFFFF */
} pic_event;

typedef struct pic_ctx pic_ctx;

/* Bytes of work memory pic_init needs for this configuration and these
 * capacities (cap[3] particles per species). */
pic_status pic_scratch_size(const pic_config* cfg, const int64_t cap[3], size_t* bytes);

/* Create a context: the statement of the problem of Sec. 2.1 (Eq. poi with
 * the boundary conditions bcf1-bcf3) on the node grid. Validates cfg
 * (INVALID_ARG), computes the node types (0 V on the cathode plane and inside
 * or on the tip, V0 on the anode plane, zero normal field on the lateral
 * faces), solves the unit-anode Laplace problem to cfg->laplace_rtol (phi1,
 * and its field field0, the weighting field of the Shockley-Ramo current of
 * Sec. 2.3.1), sets V0 = apex_field / (Laplace apex field per volt),
 * phi = V0 phi1 and the node field, and empties all species. bufs and the
 * stream are borrowed, not owned. Synchronizes the stream. Errors:
 * INVALID_ARG (config, NULL or misaligned buffers, scratch too small), HIP,
 * NOT_CONVERGED (Laplace solve). */
pic_status pic_init(const pic_config* cfg, const pic_buffers* bufs, void* hip_stream, pic_ctx** out);

/* With src != NULL: append src->n particles of one species (copied from
 * device memory), numbering them from the next id in array order.
 * With src == NULL: the surface injection of the current step (as
 * PIC_STEP_INJECT): Fowler-Nordheim emission, then evaporation when
 * cfg.surface_T > 0. n_added (optional) receives the number appended; the
 * call synchronizes. Errors: INVALID_ARG, CAPACITY. */
pic_status pic_inject(pic_ctx* ctx, const pic_particles* src, int64_t* n_added);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): the Fowler-Nordheim
 * emission of pic_inject(ctx, NULL, n_added), with the same result, whose
 * work memory (the per-patch counts and per-block sums) is a static device
 * array of 1 MiB held by each GPU the library runs on until the process ends,
 * instead of the context's scratch. The caller still owns the particle
 * arrays that receive the electrons. Allocates nothing. Every call on one GPU
 * shares that GPU's array and leaves its contents behind (every entry a call
 * reads is written earlier in the same call, so none needs clearing); calls
 * that overlap on one GPU, from any context or stream, race. Errors:
 * INVALID_ARG when the emission needs more than 1 MiB of work memory (about
 * 260 000 patches), CAPACITY, STATE. Synchronizes the stream. */
pic_status pic_inject_noalloc(pic_ctx* ctx, int64_t* n_added);

/* Run nsteps steps of the phases selected in flags (PIC_STEP_*). The
 * work is enqueued on the stream; only the solve phase synchronizes (to test
 * convergence). */
pic_status pic_step(pic_ctx* ctx, int32_t nsteps, uint32_t flags);

/* Solve Eq. poi (Sec. 2.1, with bcf1-bcf3) for the charge in rho with the
 * given solver and guess until ||b - A phi|| <= rtol ||b|| or maxit
 * iterations, then compute the node field. With PIC_GUESS_LEARNED the initial
 * residual of the network's guess is compared with that of V0 phi1 first; a
 * guess that is not finite or is worse is replaced by V0 phi1 (info->fell_back),
 * so the result never depends on the network, only the iteration count does.
 * Returns NOT_CONVERGED (context stays usable) when maxit is reached. */
pic_status pic_solve_poisson(pic_ctx* ctx, int32_t solver, int32_t guess, double rtol, int32_t maxit,
                             pic_solve_info* info);

/* Observables of the current state (the particle counts and event counts
 * of Sec. 3.2, the Shockley-Ramo gap current I = sum q v . E0 of Sec. 2.3.1
 * with E0 = field0, kinetic energies, removals per boundary, emission and
 * solver statistics) by fixed-order reductions, copied to the caller's host
 * struct. Synchronizes the stream and reports sticky device errors
 * (CAPACITY, OVERFLOW), after which the context is in a failed state. */
pic_status pic_moments(pic_ctx* ctx, pic_moments_t* out);

/* Copy up to cap events of the last collide phase run with PIC_STEP_EVENTS;
 * n receives the number recorded. */
pic_status pic_events(pic_ctx* ctx, pic_event* out, int64_t cap, int64_t* n);

/* Timers. With profiling enabled, pic_step and pic_solve_poisson record HIP
 * events on the context stream around each phase and around the hot kernels
 * (the kernels of the first 64 solver iterations of each solve), and the
 * multigrid solver launches its iterations one by one instead of as a
 * captured graph; pic_timers adds up the elapsed times since the last reset
 * (synchronizes). */
#define PIC_T_INJECT 0        /* emission phase */
#define PIC_T_PUSH_E 1        /* electron push kernel (gather, push, deposit, binning) */
#define PIC_T_PUSH 2          /* the three push kernels */
#define PIC_T_PARTICLES 3     /* push phase: clearing of rho and counters, push kernels */
#define PIC_T_COLLIDE 4       /* collide phase: bins, MCC, field ionization, products, reordering */
#define PIC_T_MCC 5           /* the two MCC kernels */
#define PIC_T_SOLVE 6         /* Poisson solve and node field */
#define PIC_T_CG_A 7          /* CG kernel: p update, matrix product, p.q */
#define PIC_T_CG_B 8          /* CG kernel: x and r update, r.r */
#define PIC_T_STEP 9          /* whole steps of pic_step */
#define PIC_T_MG 10           /* multigrid V-cycles */
#define PIC_T_DEPOSIT 11      /* tiled charge deposit kernel */
#define PIC_T_BIN 12          /* cell bins (radix sort of the cell keys) */
#define PIC_T_MG_FIRST 13     /* finest-level pre-smoothing kernel (two sweeps from zero) */
#define PIC_T_MG_RESTRICT 14  /* finest-level residual kernel (input of the restriction) */
#define PIC_T_MG_CORR 15      /* finest-level prolongation of the coarse correction */
#define PIC_T_MG_LAST 16      /* finest-level last sweep kernel (with the r.z partials) */
#define PIC_NTIMERS 17

pic_status pic_profile(pic_ctx* ctx, int32_t enable);
/* ms[PIC_NTIMERS]: summed milliseconds; count[PIC_NTIMERS]: number of timed
 * intervals; reset != 0 clears the sums afterwards. */
pic_status pic_timers(pic_ctx* ctx, double* ms, int64_t* count, int32_t reset);

const char* pic_last_error(const pic_ctx* ctx);
void pic_destroy(pic_ctx* ctx);

/* ---------------------------------------------------------------------------
 * Learned warm start of the Poisson solve (an extension: the paper solves
 * Eq. poi from the previous solution; here a network supplies the guess and
 * CG to the same tolerance still decides the result, so a poor network costs
 * iterations, never accuracy).
 *
 * Normalization. With q = rho 2^-40 (elementary charges per node) and
 * s = max |q|, the network maps x = q / s to y, and the guess is
 *   phi0 = V0 phi1 + (e s / (eps0 h)) y
 * (or V0 phi1 + gamma y with the energy-norm weight gamma, see
 * pic_set_learned_guess).
 * The charge part phi_rho = phi - V0 phi1 solves A phi_rho = q e / (eps0 h)
 * with zero on every fixed node, so y* = phi_rho eps0 h / (e s) solves A y* = x:
 * the target is dimensionless and of order one whatever the charge.
 *
 * Network: a 3D U-Net on [batch][d][h][w] fp32 inputs (d = nz, h = ny,
 * w = nx, each a multiple of 8): four levels of 16, 32, 64, 128 channels, two
 * 3x3x3 convolutions with ReLU per level (zero padding), 2x2x2 stride-2
 * convolutions with ReLU down, 2x2x2 stride-2 transposed convolutions up,
 * skip connections by channel concatenation (upsampled first), and a linear
 * 1x1x1 head. Weights and activations are bf16 on the matrix cores with fp32
 * accumulation; the master parameters, gradients and Adam moments are fp32.
 *
 * Parameter vector (fp32, caller-owned device memory), layer by layer in
 * network order, each as W then b: W[tap][cin][cout] with tap = 9 dz + 3 dy
 * + dx (offsets -1..1) for the 3x3x3 convolutions and tap = 4 pz + 2 py + px
 * (0..1) for the down convolutions (input voxel 2v + p) and the transposed
 * convolutions (output voxel 2v + p); a concatenating layer takes the
 * upsampled tensor as its first cin channels. The first layer reads 8 input
 * channels of which only channel 0 carries x (the others are zero). The head
 * is w[16] then b[1]. */
typedef struct pic_unet_config {
    int32_t base_channels; /* must be 16 */
    int32_t reserved[7];
} pic_unet_config;

typedef struct unet unet;

/* Number of fp32 parameters. */
pic_status unet_param_count(const pic_unet_config* cfg, int64_t* n);
/* Bytes of device work memory for a network over batch x d x h x w inputs
 * (d, h, w multiples of 8, at least 8; batch d h w below 2^31).
 * INVALID_ARG otherwise. */
pic_status unet_workspace_size(const pic_unet_config* cfg, int32_t batch, int32_t d, int32_t h, int32_t w,
                               size_t* bytes);
/* Create a network over caller-owned device memory: params and grads hold
 * unet_param_count floats each, workspace (256-byte aligned) at least
 * unet_workspace_size bytes. The parameters are read now and after every
 * unet_adam_step / unet_sync_params. All work goes to hip_stream. */
pic_status unet_create(const pic_unet_config* cfg, float* params, float* grads, void* workspace, size_t ws_bytes,
                       int32_t batch, int32_t d, int32_t h, int32_t w, void* hip_stream, unet** out);
/* y = net(x); x, y device fp32 [batch][d][h][w] (y may be NULL: the output
 * stays inside the workspace for unet_backward). */
pic_status unet_forward(unet* net, const float* x, float* y);
/* Gradients of the mean squared error between the last forward output and
 * target (device fp32, same shape) into grads (overwritten). loss (optional,
 * host) receives the loss and makes the call synchronize. */
pic_status unet_backward(unet* net, const float* target, double* loss);
/* One Adam step (bias-corrected) on params with grads; refreshes the bf16
 * weights. */
pic_status unet_adam_step(unet* net, float lr, float beta1, float beta2, float eps);
/* Re-read params after the caller changed them. */
pic_status unet_sync_params(unet* net);
void unet_destroy(unet* net);

/* Use net (created with batch 1 over nz x ny x nx on the context's stream)
 * for PIC_GUESS_LEARNED; NULL detaches. The network must outlive its use.
 * smooth_passes (0..64) binomial [1 2 1]/4 filters along x, y and z are
 * applied to the network output y before it enters the guess
 * V0 phi1 + gamma y (free nodes). project = 0: gamma = e s / (eps0 h), the
 * network's own scale; project = 1: gamma = (y.q) / (y.L y), q the charge
 * term and L the operator of Eq. poi, the weight that minimizes the energy
 * norm of the error along y (the guess is then never worse in that norm than
 * V0 phi1; one extra pass over the grid). fallback = 1: plain CG judges the
 * guess before every solve (the initial residuals of the guess and of V0 phi1,
 * one residual pass each) and starts from V0 phi1 instead when the network's
 * guess is not finite or has the larger residual (pic_solve_info.fell_back);
 * fallback = 0: the network's guess is used as it is (for inspecting it).
 * Invalid arguments: PIC_E_INVALID_ARG. */
pic_status pic_set_learned_guess(pic_ctx* ctx, unet* net, int32_t smooth_passes, int32_t project,
                                 int32_t fallback);
/* A training pair from the current state: x = q / s from rho and
 * y = (phi - V0 phi1) eps0 h / (e s) from phi (solve to a tight tolerance
 * first). x, y: device fp32 [nz][ny][nx]; scale (optional, host) receives s
 * (synchronizes). A state without charge gives x = y = 0 and s = 0. */
pic_status pic_training_sample(pic_ctx* ctx, float* x, float* y, double* scale);

#ifdef __cplusplus
}
#endif
#endif
