/*
 * oracle.h -- plain FP64 CPU oracle of the electrostatic PIC-MCC step of
 * "Simulating vacuum arc initiation by coupling emission, heating and plasma
 * processes" (arXiv 2402.08404).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may include, link or
 * call this code; it exists so that tests and the CPU baseline can check the
 * GPU library against a slow, obviously correct implementation. It shares no
 * code, header, constant or table generator with the GPU library.
 *
 * Units and state (a reading of Sec. 2.2, where the paper gives SI physics):
 *   - positions are stored in grid units X = x/h, node (i,j,k) sits at X=i;
 *   - velocities are stored in grid units per step V = v*dt/h;
 *   - all physics below converts to SI where a formula needs it.
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H
#include <stdint.h>

typedef struct orc_config {
    int32_t nx, ny, nz, xs_n;
    double h;            /* node spacing [m] */
    double tip_r;        /* tip radius [m] */
    double tip_h;        /* total tip height to the apex [m] */
    double dt;           /* time step [s] */
    double phi_w;        /* work function [eV] */
    double xi;           /* first ionization energy of Cu [eV] */
    double m_ion;        /* Cu mass [kg] */
    double xs_emin;      /* first table node energy [eV] */
    double xs_emax;      /* last table node energy [eV] */
    const double* xs_el; /* e-Cu elastic cross section [m^2] at xs_n log nodes */
    const double* xs_iz; /* e-Cu impact ionization cross section [m^2] */
    const double* xs_cx; /* Cu+-Cu charge exchange cross section [m^2] */
    uint64_t seed;       /* Philox key */
    int32_t fn_rings;    /* cap rings of emission patches */
    int32_t fn_az;       /* azimuthal patches per ring */
    int32_t w_max;       /* largest superparticle weight of evaporated neutrals (<= 1: all weights 1) */
    int32_t pad;
    double n_max;        /* SP number density [1/m^3] above which evaporated neutrals get heavier */
    double sigma_nn;     /* Cu-Cu elastic (hard-sphere) cross section [m^2] */
    double coulomb_log;  /* Coulomb logarithm ln(Lambda) of the Takizuka-Abe collisions */
    double sigma_rec;    /* Cu+ + e -> Cu recombination cross section [m^2] */
} orc_config;

/* Superparticle weights (Sec. 2.3.2): w[p] physical particles per SP, in
 * units of the smallest weight w_min = 1 (NULL: every weight is 1). */
typedef struct orc_species {
    int64_t n, cap;
    double *x, *y, *z, *vx, *vy, *vz;
    uint32_t* id;
    uint32_t* w;
} orc_species;

typedef struct orc_event {
    int32_t kind;   /* 1 elastic e-Cu, 2 impact ionization, 3 charge exchange, 4 field ionization */
    uint32_t id_a;  /* electron (kinds 1,2) or ion (kind 3); UINT32_MAX for kind 4 */
    uint32_t id_b;  /* the neutral */
    uint32_t new_ion, new_e; /* ids of the products (kinds 2,4), else UINT32_MAX */
} orc_event;

typedef struct orc_collide_out {
    orc_event* ev; int64_t ev_cap, n_ev;
    uint32_t* fragile; int64_t fr_cap, n_fragile;
    int64_t n_kind[5];
    int64_t n_bsi_skip;     /* neutrals above the barrier-suppression limit */
    int64_t n_kind_w[5];    /* physical collisions per kind (sum of N_coll over the events) */
    int64_t n_split;        /* superparticles split off by partial collisions */
    int64_t n_nn;           /* Cu-Cu elastic collisions */
    int64_t n_coul;         /* Coulomb scatterings (pairs with u > 0) */
    int64_t n_rec;          /* recombinations */
} orc_collide_out;

enum { ORC_SP_E = 0, ORC_SP_ION = 1, ORC_SP_NEU = 2 };
enum { ORC_ALIVE = 0, ORC_CATHODE = 1, ORC_ANODE = 2, ORC_LATERAL = 3, ORC_TIP = 4 };
enum { ORC_FREE = 0, ORC_DIR0 = 1, ORC_DIRV = 2 };
enum { ORC_COLL_MCC1 = 1, ORC_COLL_MCC2 = 2, ORC_COLL_FI = 4, ORC_COLL_NN = 8, ORC_COLL_COUL = 16, ORC_COLL_REC = 32 };

void orc_constants(double out[8]);
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_uniform(uint32_t hi, uint32_t lo);

int orc_inside_tip(const orc_config* c, double X, double Y, double Z);
void orc_node_types(const orc_config* c, uint8_t* type);
void orc_rhs(const orc_config* c, const uint8_t* type, const int64_t* Q, double V0, double* b);
void orc_apply_A(const orc_config* c, const uint8_t* type, const double* x, double* y);
int orc_solve(const orc_config* c, const uint8_t* type, const int64_t* Q, double V0,
              double* phi, double rtol, int maxit, double* relres);
void orc_field(const orc_config* c, const double* phi, double* E);
void orc_gather(const orc_config* c, const double* E, double X, double Y, double Z, double out[3]);
double orc_interp_phi(const orc_config* c, const double* phi, double X, double Y, double Z);
double orc_apex_field(const orc_config* c, const double* phi1);

void orc_push(const orc_config* c, const double* E, orc_species* s, double q, double m,
              int32_t* code);
void orc_push_sr(const orc_config* c, const double* E, const double* E0, orc_species* s, double q, double m,
                 int32_t* code, double* isr);
void orc_deposit(const orc_config* c, const orc_species* s, int64_t sign, int64_t* Q);
int64_t orc_cell_of(const orc_config* c, double X, double Y, double Z);

double orc_xs(const orc_config* c, const double* tab, double E);
double orc_adk_rate(const orc_config* c, double E_GVm);
double orc_fn_current(const orc_config* c, double F, int* clamped);
int64_t orc_fn_patch_count(const orc_config* c);
void orc_fn_patch(const orc_config* c, int64_t p, double ua, double ub, double out[8]);
int64_t orc_fn_inject(const orc_config* c, uint32_t step, const double* phi, orc_species* e,
                      uint32_t* next_id, double* n_expected, int64_t* n_clamped);

double orc_evap_flux(const orc_config* c, double T);
int64_t orc_evaporate(const orc_config* c, uint32_t step, double T, orc_species* nsp, uint32_t* next_id,
                      double* n_expected, const int64_t* cell_count);

int orc_collide(const orc_config* c, uint32_t step, int32_t flags, const double* E,
                orc_species* sp, uint32_t* next_id, orc_collide_out* out);

void orc_moments(const orc_config* c, const orc_species* sp, const double* E0, double out[8]);
#endif
