/* pic_rz.h -- C ABI of the 2D axisymmetric (r, z) 2D3V variant of the
 * particle-mesh step (Sec. 2.2: an axisymmetric vacuum mesh around the tip,
 * three velocity components with the azimuthal one kept, particles rotated
 * back into the r-z plane every step, reflection at the axis, removal at the
 * cathode, the anode and the open side, leapfrog integration).
 *
 * Scope: the node grid with its tip, Poisson's equation in cylindrical
 * finite-volume form solved by FP64 conjugate gradients preconditioned by a
 * geometric multigrid V-cycle, the node field, the gather, push, rotation
 * and removal of electrons, Cu+ (and Cu2+) ions and Cu neutrals, the fixed-point charge deposit, the pair collisions of Table
 * colls (elastic e-Cu, impact ionization, charge exchange Cu+-Cu, and with
 * cu2 the double ionization of Cu and the ionization of Cu+; Eqs. colp, du,
 * newv), field ionization of Cu (Eq. dfi) and Fowler-Nordheim emission
 * (Sec. 2.3.1). Superparticle weights, same-species and Coulomb collisions,
 * recombination, evaporation and the circuit of the 3D library are not part
 * of this variant.
 *
 * Discretization: nodes at (r, z) = (i h, k h), 0 <= i < nr, 0 <= k < nz,
 * node n = k * nr + i. Nodes of the plane k = 0 and inside the tip (a
 * cylinder of radius tip_r on the axis up to tip_h - tip_r, a hemisphere on
 * top) are held at 0 V, k = nz - 1 at V0; the side r = (nr - 1) h has zero
 * normal field. For a free node, with annular control volumes r in
 * [r_i - h/2, r_i + h/2] clipped to [0, (nr - 1) h]:
 *     sum_j c_ij (phi_i - phi_j) = Q_i / (pi eps0 h),
 * couplings c = 2 (i - 1/2) and 2 (i + 1/2) through the radial faces (none
 * through the axis or the side), (r_hi^2 - r_lo^2) / h^2 through each axial
 * face. V0 = apex_field / F1 with F1 = phi1(0, tip_h + h) / h from the
 * unit-anode solution phi1 (as in the 3D library).
 *
 * Particles (per species 0 electrons, 1 Cu+, 2 Cu): r, z in grid units
 * (r / h, z / h), vr, vt, vz (radial, azimuthal, axial) in grid units per
 * step (v dt / h), uint32 ids (0xFFFFFFFF: a free slot). One push: the kick
 * of (vr, vz) by the bilinearly gathered node field (E_r = 0 on the axis and
 * on the side), the drift x = r + vr, y = vt, z += vz in the particle's own
 * Cartesian frame, then r' = sqrt(x^2 + y^2) and (vr, vt) turned by the
 * angle atan2(y, x); removal (the slot's id set free) at z <= 0, z >=
 * nz - 1, r' >= nr - 1 or inside the tip. Deposit: bilinear weights per axis
 * quantized to 2^-20, every particle adds exactly 2^40 units of 2^-40 e.
 *
 * Collisions (PIC_RZ_COLLIDE), in the 3D library's pairing: the cell (i, k)
 * lies between the nodes i, i + 1 and k, k + 1 (key k (nr - 1) + i, the
 * per-cell draw's counter); the particles of a species in a cell, in
 * ascending id order, pair with the other species' as in pic.h (the smaller
 * count projects, targets shifted cyclically by floor(U_c N_t)); the density
 * is N_t / (pi (2 i + 1) h^3), the annular cell volume; (v_r, v_theta, v_z)
 * enter as Cartesian components. (e, Cu) first, then (Cu+, Cu) without the
 * neutrals that had an event; then field ionization of the remaining
 * neutrals below the barrier-suppression field 1.5 xi^1.5 GV/m; then the
 * products, impact ionizations before field ionizations, each in ascending
 * neutral id; each product's new ion (if any) takes the next id and the
 * next ion slot, its new electrons the following ids and the next electron
 * slots; the ionized neutral's slot is freed. With cu2 the ions carry a
 * charge state (1 or 2; kick and deposit scale with it): the (e, Cu) class
 * has a third process, Cu + e -> Cu2+ + 3e above xi + xi2 (the energy above
 * it shared by the three electrons as U5, U6 (1 - U5) and the rest, draws
 * 1 to 4 of the pair), and a third class pairs electrons with ions after
 * the (Cu+, Cu) class: Cu+ + e -> Cu2+ + 2e above xi2 (draw tags 36 for the
 * cell shift, 37 for the pair), the ion keeping its slot, id and velocity;
 * particles with an event this step and Cu2+ ions sit out; these products
 * come after the field ionizations, in ascending ion id, one new electron
 * each. Emission (PIC_RZ_EMIT): fn_rings equal-area
 * rings of the cap, then rings one spacing high on the cylinder, each with
 * the Murphy-Good current J at the field phi(s + n) / h one spacing out
 * along the normal from its mid point s; N = J A h^2 dt / e electrons, floor(N)
 * plus one with probability frac(N) (draw (patch, step, 6, 0)); electron j
 * at ring parameter U from draw (patch, step, 6, 1 + j), 10^-3 spacings out,
 * at rest; ids continue from next_id in patch order. New particles are
 * appended at the end of the species' slots. Ids must be unique and not
 * 0xFFFFFFFF; the pairing and the products follow the ids, not the slots.
 */
#ifndef PIC_RZ_H
#define PIC_RZ_H
#include <stddef.h>
#include <stdint.h>

#include "pic.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pic_rz_config {
    int32_t nr, nz;        /* nodes along r and z, nr >= 4, nz >= 4 */
    double h;              /* node spacing [m] */
    double tip_r;          /* tip radius [m] (0: no tip) */
    double tip_h;          /* total tip height to the apex [m] */
    double apex_field;     /* Laplace field just above the apex [V/m] */
    double dt;             /* time step [s] */
    double m_ion;          /* Cu mass [kg] */
    double laplace_rtol;   /* tolerance of the unit-anode solve at init */
    int32_t maxit;         /* iteration limit of the solve inside pic_rz_step */
    int32_t sort_every;    /* with collisions: every this many steps (0: never) the particles of
                              each species are reordered by cell, ascending id within a cell,
                              freed slots dropped (slots change, ids stay) */
    double step_rtol;      /* tolerance of the solve inside pic_rz_step */
    /* collisions, field ionization, emission */
    uint64_t seed;         /* Philox key of every draw */
    double xi;             /* ionization energy of Cu [eV] */
    double phi_w;          /* work function [eV] */
    double xs_emin, xs_emax; /* energy range of the cross-section tables [eV], log-spaced */
    int32_t xs_n;          /* table length, >= 2 (0: no tables; PIC_RZ_COLLIDE then fails) */
    int32_t fn_rings;      /* rings on the cap (0: no emission; PIC_RZ_EMIT then fails) */
    /* Cu2+ (Table colls: Cu + e -> Cu2+ + 3e, Cu+ + e -> Cu2+ + 2e) as the
     * charge state of an ion; 0: every ion is Cu+ */
    int32_t cu2;
    int32_t reserved3;
    double xi2;            /* second ionization energy of Cu [eV] */
} pic_rz_config;

typedef struct pic_rz_buffers {
    /* per species s: arrays of capacity cap[s] (device memory, FP64); the
     * first n[s] slots hold the initial particles when pic_rz_init is called */
    double* r[3];
    double* z[3];
    double* vr[3];
    double* vt[3];
    double* vz[3];
    uint32_t* id[3];
    int64_t cap[3];
    int64_t n[3];
    double* phi;           /* nr*nz potential [V] */
    double* phi1;          /* nr*nz unit-anode potential, written by pic_rz_init */
    int64_t* rho;          /* nr*nz node charge [2^-40 e] */
    double* field;         /* 2*nr*nz node field (E_r, E_z) [V/m] */
    uint8_t* node_type;    /* nr*nz: 0 free, 1 held at 0 V, 2 held at V0 */
    void* scratch;         /* pic_rz_scratch_size bytes, 256-byte aligned */
    size_t scratch_bytes;
    const double* xs;      /* 3 * xs_n cross sections [m^2] (5 * xs_n with cu2): elastic,
                              ionization, charge exchange (, double ionization of Cu,
                              ionization of Cu+) at xs_emin (xs_emax / xs_emin)^(k / (xs_n - 1)),
                              all >= 0 */
    uint8_t* charge;       /* with cu2: cap[1] charge states of the ions (1 or 2; the first
                              n[1] given at pic_rz_init), kept by the library */
} pic_rz_buffers;

typedef struct pic_rz_moments_t {
    int64_t n_alive[3];      /* alive particles per species */
    int64_t absorbed[3][5];  /* cumulative removals: 1 cathode, 2 anode, 3 side, 4 tip */
    int64_t q_total;         /* sum of rho [2^-40 e] */
    int64_t step;            /* step counter */
    double v0;               /* anode potential [V] */
    double apex_field1;      /* F1, apex field per volt of anode potential [1/m] */
    int32_t last_cg_iters;   /* iterations of the last solve */
    int32_t error;           /* sticky error code */
    int64_t n_slots[3];      /* slots in use per species (alive and freed) */
    int64_t events[5];       /* cumulative: 1 elastic, 2 impact ionization, 3 charge exchange, 4 field ionization */
    int64_t injected;        /* cumulative emitted electrons */
    int64_t next_id;         /* id of the next new particle */
    int64_t double_ionizations; /* cumulative Cu + e -> Cu2+ + 3e */
    int64_t ion_ionizations;    /* cumulative Cu+ + e -> Cu2+ + 2e */
    int64_t n_cu2;              /* alive ions of charge state 2 */
} pic_rz_moments_t;

typedef struct pic_rz_ctx pic_rz_ctx;

/* flags of pic_rz_step */
#define PIC_RZ_PUSH 1u     /* gather, push, rotation, removal */
#define PIC_RZ_DEPOSIT 2u  /* charge deposit into rho */
#define PIC_RZ_SOLVE 4u    /* Poisson solve to step_rtol from the previous potential, then the node field */
#define PIC_RZ_ADVANCE 8u  /* count the step */
#define PIC_RZ_FIELD 16u   /* without PIC_RZ_SOLVE: the node field of the current phi */
#define PIC_RZ_EMIT 32u    /* field emission (before the push) */
#define PIC_RZ_COLLIDE 64u /* collisions, field ionization, products (after the push) */
#define PIC_RZ_FULL 15u
#define PIC_RZ_ALL 111u    /* PIC_RZ_FULL with emission and collisions */

/* Bytes of work memory for cfg and cap. Invalid config: PIC_E_INVALID_ARG. */
pic_status pic_rz_scratch_size(const pic_rz_config* cfg, const int64_t cap[3], size_t* bytes);

/* Create a context on hip_stream (NULL: the default stream): node types, the
 * unit-anode solve (to laplace_rtol) into phi1, V0, phi = V0 phi1 and its
 * field; next_id = one above the largest initial id (0 without particles).
 * Buffers are caller-owned; the context keeps their pointers.
 * Errors: PIC_E_INVALID_ARG (config, buffers, n > cap, an initial id
 * 0xFFFFFFFF, a charge state other than 1 or 2), PIC_E_NOT_CONVERGED,
 * PIC_E_HIP. */
pic_status pic_rz_init(const pic_rz_config* cfg, const pic_rz_buffers* bufs, void* hip_stream, pic_rz_ctx** out);

/* nsteps steps of the stages in flags, in the order emission, push,
 * collisions, deposit, solve. Draws are keyed by the step counter, which
 * PIC_RZ_ADVANCE counts. New particles that would overflow a species'
 * capacity, or ids that would reach 0xFFFFFFFF, are not made: the stage
 * sets the sticky error and the call returns PIC_E_CAPACITY (or
 * PIC_E_OVERFLOW for ids) after its steps. PIC_E_INVALID_ARG for
 * PIC_RZ_COLLIDE without tables or PIC_RZ_EMIT without rings. */
pic_status pic_rz_step(pic_rz_ctx* ctx, int32_t nsteps, uint32_t flags);

/* Solve for the charge in rho from the current phi until ||b - A phi|| <=
 * rtol ||b|| (b with the held values moved to the right-hand side), then the
 * node field. info may be NULL. PIC_E_NOT_CONVERGED if maxit is reached. */
pic_status pic_rz_solve(pic_rz_ctx* ctx, double rtol, int32_t maxit, pic_solve_info* info);

/* Synchronizes the stream and reports counts and the sticky error. */
pic_status pic_rz_moments(pic_rz_ctx* ctx, pic_rz_moments_t* out);

const char* pic_rz_last_error(const pic_rz_ctx* ctx);
void pic_rz_destroy(pic_rz_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
