/*
 * oracle.c -- plain FP64 CPU oracle of the electrostatic PIC-MCC step of
 * arXiv 2402.08404 ("Simulating vacuum arc initiation by coupling emission,
 * heating and plasma processes").
 *
 * TEST INFRASTRUCTURE ONLY: only tests/, the smoke check and the CPU baseline
 * of bench.py may load this library. It is deliberately slow and literal:
 * single-threaded loops, no blocking, no fusion, each function following the
 * passage it cites. Build flags: -O2 -ffp-contract=off -fno-fast-math.
 *
 * Every reading of a passage the paper leaves silent or ambiguous is stated
 * where it is used.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* CODATA 2022 values (SI). */
#define E_CH 1.602176634e-19     /* elementary charge [C] */
#define M_EL 9.1093837139e-31    /* electron mass [kg] */
#define EPS0 8.8541878188e-12    /* vacuum permittivity [F/m] */
#define H_PL 6.62607015e-34      /* Planck constant [J s] */
#define AMU 1.66053906892e-27    /* atomic mass constant [kg] */
#define PI 3.14159265358979323846

/* Philox counter tags: the third counter word names the purpose of a draw. */
#define TAG_MCC1 1u
#define TAG_MCC2 2u
#define TAG_PAIR1 3u
#define TAG_PAIR2 4u
#define TAG_FI 5u
#define TAG_INJ 6u

/* Weight of superparticle p (Sec. 2.3.2), 1 without a weight array. */
static uint32_t wgt(const orc_species* s, int64_t p) { return s->w ? s->w[p] : 1u; }

/* Relative band inside which two correct libm implementations may disagree on
 * a decision U < P; decisions that close are reported as fragile. */
#define FRAGILE_REL 1.4210854715202004e-14 /* 2^-46 */
#define FRAGILE_FI 1.0e-5

/* ------------------------------------------------------------------------ */
/* Constants used by the emission model: the Fowler-Nordheim constants of the
 * Murphy-Good current density (Sec. 2.3.1 names emission from the cathode
 * surface; the closed form is the standard Murphy-Good / Forbes one). */
static double fn_a(void) { return E_CH * E_CH / (8.0 * PI * H_PL); }            /* A eV V^-2 */
static double fn_b(void) {                                                       /* eV^-3/2 V/m */
    return (8.0 * PI / 3.0) * sqrt(2.0 * M_EL) / (E_CH * H_PL) * pow(E_CH, 1.5);
}
static double fn_cs2(void) { return E_CH / (4.0 * PI * EPS0); }                 /* eV^2 m/V */

void orc_constants(double out[8]) {
    out[0] = E_CH; out[1] = M_EL; out[2] = EPS0; out[3] = H_PL; out[4] = AMU;
    out[5] = fn_a(); out[6] = fn_b(); out[7] = fn_cs2();
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
 * multiplies with xor mixing, the key bumped by the Weyl constants between
 * rounds. Written from the published description. */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* A uniform in (0,1) from 52 random bits: (k + 1/2) 2^-52, exact in FP64. */
double orc_uniform(uint32_t hi, uint32_t lo) {
    uint64_t k = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
    return ((double)k + 0.5) * 0x1p-52;
}

static void draw2(const orc_config* c, uint32_t a, uint32_t step, uint32_t tag, uint32_t sub,
                  double* u0, double* u1) {
    uint32_t ctr[4] = {a, step, tag, sub};
    uint32_t key[2] = {(uint32_t)c->seed, (uint32_t)(c->seed >> 32)};
    uint32_t w[4];
    orc_philox(ctr, key, w);
    *u0 = orc_uniform(w[0], w[1]);
    *u1 = orc_uniform(w[2], w[3]);
}

/* ------------------------------------------------------------------------ */
/* Geometry (Sec. 2.1, boundary conditions bcf1-bcf3). Reading: a 3D box of
 * nodes; the cathode plane z=0 and a Cu tip standing on it at the box centre
 * (cylinder of radius r up to z = H - r, hemispherical cap reaching z = H)
 * are held at 0 V; the anode plane z = (nz-1)h is held at V0; the four lateral
 * faces are the vacuum boundary with zero normal field. */
int orc_inside_tip(const orc_config* c, double X, double Y, double Z) {
    double R = c->tip_r / c->h;
    double H = c->tip_h / c->h;
    double zc = H - R;
    double xc = 0.5 * (double)(c->nx - 1);
    double yc = 0.5 * (double)(c->ny - 1);
    double dx = X - xc, dy = Y - yc;
    double rho2 = dx * dx + dy * dy;
    if (Z < 0.0) return 0;
    if (Z <= zc) return rho2 <= R * R;
    double dz = Z - zc;
    return rho2 + dz * dz <= R * R;
}

void orc_node_types(const orc_config* c, uint8_t* type) {
    for (int k = 0; k < c->nz; ++k)
        for (int j = 0; j < c->ny; ++j)
            for (int i = 0; i < c->nx; ++i) {
                int64_t n = ((int64_t)k * c->ny + j) * c->nx + i;
                if (k == 0) type[n] = ORC_DIR0;
                else if (k == c->nz - 1) type[n] = ORC_DIRV;
                else if (orc_inside_tip(c, i, j, k)) type[n] = ORC_DIR0;
                else type[n] = ORC_FREE;
            }
}

/* ------------------------------------------------------------------------ */
/* Poisson's equation (Sec. 2.1, Eq. poi) in finite-volume form on node control
 * volumes clipped at the lateral faces: for a free node i,
 *     sum_j f_ij (phi_i - phi_j) = q_i / (eps0 h),
 * where f_ij is the fraction of a full h^2 face shared by i and j (1 inside,
 * 1/2 on a lateral face, 1/4 on a lateral edge) and q_i the node charge. The
 * zero normal-field condition (bcf2) is the absence of flux through the
 * lateral faces; Dirichlet values enter the right-hand side. */
static double half_at_edge(int i, int n) { return (i == 0 || i == n - 1) ? 0.5 : 1.0; }

static double dirichlet_value(uint8_t t, double V0) { return t == ORC_DIRV ? V0 : 0.0; }

void orc_rhs(const orc_config* c, const uint8_t* type, const int64_t* Q, double V0, double* b) {
    int nx = c->nx, ny = c->ny, nz = c->nz;
    double qscale = ldexp(1.0, -40) * E_CH / (EPS0 * c->h);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int64_t n = ((int64_t)k * ny + j) * nx + i;
                if (type[n] != ORC_FREE) { b[n] = 0.0; continue; }
                double s = (double)Q[n] * qscale;
                double fx = half_at_edge(j, ny) * half_at_edge(k, nz);
                double fy = half_at_edge(i, nx) * half_at_edge(k, nz);
                double fz = half_at_edge(i, nx) * half_at_edge(j, ny);
                if (i > 0 && type[n - 1] != ORC_FREE) s += fx * dirichlet_value(type[n - 1], V0);
                if (i < nx - 1 && type[n + 1] != ORC_FREE) s += fx * dirichlet_value(type[n + 1], V0);
                if (j > 0 && type[n - nx] != ORC_FREE) s += fy * dirichlet_value(type[n - nx], V0);
                if (j < ny - 1 && type[n + nx] != ORC_FREE) s += fy * dirichlet_value(type[n + nx], V0);
                int64_t pl = (int64_t)nx * ny;
                if (type[n - pl] != ORC_FREE) s += fz * dirichlet_value(type[n - pl], V0);
                if (type[n + pl] != ORC_FREE) s += fz * dirichlet_value(type[n + pl], V0);
                b[n] = s;
            }
}

/* y = A x on the free nodes; Dirichlet entries of x are treated as zero. */
void orc_apply_A(const orc_config* c, const uint8_t* type, const double* x, double* y) {
    int nx = c->nx, ny = c->ny, nz = c->nz;
    int64_t pl = (int64_t)nx * ny;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int64_t n = ((int64_t)k * ny + j) * nx + i;
                if (type[n] != ORC_FREE) { y[n] = 0.0; continue; }
                double fx = half_at_edge(j, ny) * half_at_edge(k, nz);
                double fy = half_at_edge(i, nx) * half_at_edge(k, nz);
                double fz = half_at_edge(i, nx) * half_at_edge(j, ny);
                double s = 0.0;
#define NB(m, f) s += (f) * (x[n] - (type[m] == ORC_FREE ? x[m] : 0.0))
                if (i > 0) NB(n - 1, fx);
                if (i < nx - 1) NB(n + 1, fx);
                if (j > 0) NB(n - nx, fy);
                if (j < ny - 1) NB(n + nx, fy);
                NB(n - pl, fz);
                NB(n + pl, fz);
#undef NB
                y[n] = s;
            }
}

static double dot_free(int64_t N, const uint8_t* type, const double* a, const double* b) {
    double s = 0.0;
    for (int64_t n = 0; n < N; ++n)
        if (type[n] == ORC_FREE) s += a[n] * b[n];
    return s;
}

/* Plain conjugate gradients (Hestenes-Stiefel) on the free nodes. phi holds
 * the initial guess on entry (its free entries) and the full potential,
 * Dirichlet values included, on exit. Stops when ||b - A phi|| <= rtol ||b||
 * (recursively updated residual). Returns the number of matrix products. */
int orc_solve(const orc_config* c, const uint8_t* type, const int64_t* Q, double V0,
              double* phi, double rtol, int maxit, double* relres) {
    int64_t N = (int64_t)c->nx * c->ny * c->nz;
    double* b = malloc(N * sizeof(double));
    double* r = malloc(N * sizeof(double));
    double* p = malloc(N * sizeof(double));
    double* q = malloc(N * sizeof(double));
    orc_rhs(c, type, Q, V0, b);
    for (int64_t n = 0; n < N; ++n)
        if (type[n] != ORC_FREE) phi[n] = 0.0;
    orc_apply_A(c, type, phi, q);
    for (int64_t n = 0; n < N; ++n) { r[n] = b[n] - q[n]; p[n] = r[n]; }
    double bnorm = sqrt(dot_free(N, type, b, b));
    double rr = dot_free(N, type, r, r);
    int it = 0;
    if (bnorm == 0.0) {
        for (int64_t n = 0; n < N; ++n) phi[n] = 0.0;
        rr = 0.0;
        bnorm = 1.0;
    } else {
        while (it < maxit && sqrt(rr) > rtol * bnorm) {
            orc_apply_A(c, type, p, q);
            double alpha = rr / dot_free(N, type, p, q);
            for (int64_t n = 0; n < N; ++n) {
                if (type[n] != ORC_FREE) continue;
                phi[n] += alpha * p[n];
                r[n] -= alpha * q[n];
            }
            double rr_new = dot_free(N, type, r, r);
            double beta = rr_new / rr;
            for (int64_t n = 0; n < N; ++n) p[n] = (type[n] == ORC_FREE) ? r[n] + beta * p[n] : 0.0;
            rr = rr_new;
            ++it;
        }
    }
    for (int64_t n = 0; n < N; ++n)
        if (type[n] != ORC_FREE) phi[n] = dirichlet_value(type[n], V0);
    if (relres) *relres = sqrt(rr) / bnorm;
    free(b); free(r); free(p); free(q);
    return it;
}

/* ------------------------------------------------------------------------ */
/* Node field E = -grad(phi) [V/m]: central differences inside, zero normal
 * component on the lateral faces (bcf2), one-sided differences on the two
 * Dirichlet planes. E is stored as 3 doubles per node. */
void orc_field(const orc_config* c, const double* phi, double* E) {
    int nx = c->nx, ny = c->ny, nz = c->nz;
    int64_t pl = (int64_t)nx * ny;
    double h = c->h;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int64_t n = ((int64_t)k * ny + j) * nx + i;
                double ex = 0.0, ey = 0.0, ez;
                if (i > 0 && i < nx - 1) ex = -(phi[n + 1] - phi[n - 1]) / (2.0 * h);
                if (j > 0 && j < ny - 1) ey = -(phi[n + nx] - phi[n - nx]) / (2.0 * h);
                if (k == 0) ez = -(phi[n + pl] - phi[n]) / h;
                else if (k == nz - 1) ez = -(phi[n] - phi[n - pl]) / h;
                else ez = -(phi[n + pl] - phi[n - pl]) / (2.0 * h);
                E[3 * n + 0] = ex; E[3 * n + 1] = ey; E[3 * n + 2] = ez;
            }
}

/* Cloud-in-cell (trilinear) weights of a point in its cell. */
static void cic(const orc_config* c, double X, double Y, double Z, int64_t* base, double w[8]) {
    int i = (int)floor(X), j = (int)floor(Y), k = (int)floor(Z);
    i = i < 0 ? 0 : (i > c->nx - 2 ? c->nx - 2 : i);
    j = j < 0 ? 0 : (j > c->ny - 2 ? c->ny - 2 : j);
    k = k < 0 ? 0 : (k > c->nz - 2 ? c->nz - 2 : k);
    double fx = X - i, fy = Y - j, fz = Z - k;
    for (int t = 0; t < 8; ++t) {
        double wx = (t & 1) ? fx : 1.0 - fx;
        double wy = (t & 2) ? fy : 1.0 - fy;
        double wz = (t & 4) ? fz : 1.0 - fz;
        w[t] = wx * wy * wz;
    }
    *base = ((int64_t)k * c->ny + j) * c->nx + i;
}

static int64_t corner(const orc_config* c, int64_t base, int t) {
    return base + ((t & 1) ? 1 : 0) + ((t & 2) ? c->nx : 0) + ((t & 4) ? (int64_t)c->nx * c->ny : 0);
}

void orc_gather(const orc_config* c, const double* E, double X, double Y, double Z, double out[3]) {
    int64_t base; double w[8];
    cic(c, X, Y, Z, &base, w);
    out[0] = out[1] = out[2] = 0.0;
    for (int t = 0; t < 8; ++t) {
        int64_t m = corner(c, base, t);
        out[0] += w[t] * E[3 * m + 0];
        out[1] += w[t] * E[3 * m + 1];
        out[2] += w[t] * E[3 * m + 2];
    }
}

double orc_interp_phi(const orc_config* c, const double* phi, double X, double Y, double Z) {
    int64_t base; double w[8];
    cic(c, X, Y, Z, &base, w);
    double s = 0.0;
    for (int t = 0; t < 8; ++t) s += w[t] * phi[corner(c, base, t)];
    return s;
}

/* Apex field of a potential (reading: the anode voltage is set so that the
 * field just above the apex reaches the requested local field; the field is
 * the potential one node spacing above the apex divided by that spacing). */
double orc_apex_field(const orc_config* c, const double* phi1) {
    double xc = 0.5 * (double)(c->nx - 1), yc = 0.5 * (double)(c->ny - 1);
    double H = c->tip_h / c->h;
    return orc_interp_phi(c, phi1, xc, yc, H + 1.0) / c->h;
}

/* ------------------------------------------------------------------------ */
/* Leapfrog push (Sec. 2.2: positions advanced with the leapfrog scheme; no
 * magnetic field, Sec. 2.1): v^{n+1/2} = v^{n-1/2} + (q/m) E(x^n) dt and
 * x^{n+1} = x^n + v^{n+1/2} dt; neutrals (q = 0) drift. Particles that end
 * outside the vacuum region are removed (Sec. 2.2: crossing the cathode,
 * vacuum or anode boundary); code[] receives where each one left. */
void orc_push(const orc_config* c, const double* E, orc_species* s, double q, double m,
              int32_t* code) {
    orc_push_sr(c, E, NULL, s, q, m, code, NULL);
}

/* The push, also returning (E0 != NULL) the Shockley-Ramo current of the
 * pushed particles (Sec. 2.3.1): I = sum q v . E0(r) over every particle of
 * the species alive before the push, with the new velocity v^{n+1/2} and the
 * weighting field E0 (the field of the unit-anode Laplace problem) at the
 * position x^n where the kick's field was taken (reading: the paper does not
 * fix the time level; v^{n+1/2} is the velocity of the step). */
void orc_push_sr(const orc_config* c, const double* E, const double* E0, orc_species* s, double q, double m,
                 int32_t* code, double* isr) {
    double h = c->h, dt = c->dt;
    double sr = 0.0;
    for (int64_t p = 0; p < s->n; ++p) {
        if (q != 0.0) {
            double e[3];
            orc_gather(c, E, s->x[p], s->y[p], s->z[p], e);
            double vx = s->vx[p] * h / dt, vy = s->vy[p] * h / dt, vz = s->vz[p] * h / dt;
            vx += q / m * e[0] * dt;
            vy += q / m * e[1] * dt;
            vz += q / m * e[2] * dt;
            s->vx[p] = vx * dt / h; s->vy[p] = vy * dt / h; s->vz[p] = vz * dt / h;
            if (E0) {
                double w[3];
                orc_gather(c, E0, s->x[p], s->y[p], s->z[p], w);
                sr += (double)wgt(s, p) * q * (vx * w[0] + vy * w[1] + vz * w[2]);
            }
        }
        s->x[p] += s->vx[p];
        s->y[p] += s->vy[p];
        s->z[p] += s->vz[p];
        double X = s->x[p], Y = s->y[p], Z = s->z[p];
        int32_t k = ORC_ALIVE;
        if (Z <= 0.0) k = ORC_CATHODE;
        else if (Z >= (double)(c->nz - 1)) k = ORC_ANODE;
        else if (X < 0.0 || X >= (double)(c->nx - 1) || Y < 0.0 || Y >= (double)(c->ny - 1)) k = ORC_LATERAL;
        else if (orc_inside_tip(c, X, Y, Z)) k = ORC_TIP;
        code[p] = k;
    }
    if (isr) *isr = sr;
}

/* ------------------------------------------------------------------------ */
/* Charge deposition, the source term of Eq. poi. Reading of "64-bit fixed
 * point with 2^-40 charge units": cloud-in-cell weights quantized per axis to
 * 2^-13, 2^-13 and 2^-14 (round half up), so every product of the three is an
 * integer count of 2^-40 e and the eight corners of one particle sum to 2^40
 * exactly. */
static int64_t quantize(double f, int bits) {
    double t = ldexp(f, bits);          /* exact */
    double fl = floor(t);
    int64_t qv = (int64_t)fl;
    if (t - fl >= 0.5) qv += 1;         /* t - fl is exact */
    return qv;
}

void orc_deposit(const orc_config* c, const orc_species* s, int64_t sign, int64_t* Q) {
    for (int64_t p = 0; p < s->n; ++p) {
        double X = s->x[p], Y = s->y[p], Z = s->z[p];
        int i = (int)floor(X), j = (int)floor(Y), k = (int)floor(Z);
        i = i < 0 ? 0 : (i > c->nx - 2 ? c->nx - 2 : i);
        j = j < 0 ? 0 : (j > c->ny - 2 ? c->ny - 2 : j);
        k = k < 0 ? 0 : (k > c->nz - 2 ? c->nz - 2 : k);
        int64_t qx = quantize(X - i, 13), qy = quantize(Y - j, 13), qz = quantize(Z - k, 14);
        int64_t wx[2] = {8192 - qx, qx}, wy[2] = {8192 - qy, qy}, wz[2] = {16384 - qz, qz};
        int64_t base = ((int64_t)k * c->ny + j) * c->nx + i;
        int64_t sw = sign * (int64_t)wgt(s, p);     /* a superparticle of weight w carries w charges */
        for (int t = 0; t < 8; ++t)
            Q[corner(c, base, t)] += sw * wx[t & 1] * wy[(t >> 1) & 1] * wz[(t >> 2) & 1];
    }
}

int64_t orc_cell_of(const orc_config* c, double X, double Y, double Z) {
    int i = (int)floor(X), j = (int)floor(Y), k = (int)floor(Z);
    return ((int64_t)k * (c->ny - 1) + j) * (c->nx - 1) + i;
}

/* ------------------------------------------------------------------------ */
/* Cross sections sigma(E) from tables on xs_n log-spaced energies between
 * xs_emin and xs_emax, linear in ln E between nodes, clamped outside. */
double orc_xs(const orc_config* c, const double* tab, double E) {
    int n = c->xs_n;
    if (E <= c->xs_emin) return tab[0];
    if (E >= c->xs_emax) return tab[n - 1];
    double t = log(E / c->xs_emin) / log(c->xs_emax / c->xs_emin) * (double)(n - 1);
    int k = (int)floor(t);
    if (k > n - 2) k = n - 2;
    if (k < 0) k = 0;
    double f = t - k;
    return tab[k] + f * (tab[k + 1] - tab[k]);
}

/* ADK field-ionization rate per femtosecond (Sec. 2.3.4, Eq. dfi), with
 * n = 3.69 z xi^{-1/2}, z = 1, xi in eV and the field E in GV/m. */
double orc_adk_rate(const orc_config* c, double E) {
    double xi = c->xi;
    double n = 3.69 * 1.0 / sqrt(xi);
    double x32 = pow(xi, 1.5);
    if (E <= 0.0) return 0.0;
    return 1.52 * pow(4.0, n) * xi / (n * tgamma(2.0 * n)) * pow(20.5 * x32 / E, 2.0 * n - 1.0) *
           exp(-6.83 * x32 / E);
}

/* Murphy-Good field-emission current density [A/m^2] for a local field F
 * [V/m] and work function phi_w [eV], with Forbes' approximations of the
 * Schottky-Nordheim barrier functions v(f) and t(f). f is clamped at 1 (the
 * barrier vanishes there); *clamped reports it. */
double orc_fn_current(const orc_config* c, double F, int* clamped) {
    if (clamped) *clamped = 0;
    if (F <= 0.0) return 0.0;
    double phi = c->phi_w;
    double f = fn_cs2() * F / (phi * phi);
    if (f > 1.0) { f = 1.0; if (clamped) *clamped = 1; }
    double lf = log(f);
    double v = 1.0 - f + (f / 6.0) * lf;
    double t = 1.0 + f / 9.0 - (f / 18.0) * lf;
    return fn_a() * F * F / (phi * t * t) * exp(-v * fn_b() * pow(phi, 1.5) / F);
}

/* Emission patches on the analytic tip surface (reading of Sec. 2.3.1: the
 * current at each surface location gives the number of electrons injected
 * there). The hemispherical cap is cut into fn_rings rings of equal area
 * (equal steps in cos(theta)) times fn_az azimuths; the cylinder side into
 * rings one node spacing high times fn_az azimuths. out = sample point on the
 * surface for the uniforms (ua, ub) in grid units (3), outward normal (3),
 * patch area in grid units^2, 0 for cap / 1 for side. */
int64_t orc_fn_patch_count(const orc_config* c) {
    double R = c->tip_r / c->h, H = c->tip_h / c->h;
    int64_t nside = (int64_t)ceil(H - R);
    return ((int64_t)c->fn_rings + nside) * c->fn_az;
}

void orc_fn_patch(const orc_config* c, int64_t p, double ua, double ub, double out[8]) {
    double R = c->tip_r / c->h, H = c->tip_h / c->h, zc = H - R;
    double xc = 0.5 * (double)(c->nx - 1), yc = 0.5 * (double)(c->ny - 1);
    int64_t ring = p / c->fn_az, az = p % c->fn_az;
    double ph = 2.0 * PI * ((double)az + ub) / (double)c->fn_az;
    if (ring < c->fn_rings) {
        double ct = 1.0 - ((double)ring + ua) / (double)c->fn_rings;
        double st = sqrt(1.0 - ct * ct);
        double nxv = st * cos(ph), nyv = st * sin(ph), nzv = ct;
        out[0] = xc + R * nxv; out[1] = yc + R * nyv; out[2] = zc + R * nzv;
        out[3] = nxv; out[4] = nyv; out[5] = nzv;
        out[6] = 2.0 * PI * R * R / (double)c->fn_rings / (double)c->fn_az;
        out[7] = 0.0;
    } else {
        int64_t q = ring - c->fn_rings;
        double zlo = (double)q, zhi = fmin((double)(q + 1), zc);
        double z = zlo + ua * (zhi - zlo);
        double nxv = cos(ph), nyv = sin(ph);
        out[0] = xc + R * nxv; out[1] = yc + R * nyv; out[2] = z;
        out[3] = nxv; out[4] = nyv; out[5] = 0.0;
        out[6] = 2.0 * PI * R * (zhi - zlo) / (double)c->fn_az;
        out[7] = 1.0;
    }
}

static int grow_ok(const orc_species* s, int64_t extra) { return s->n + extra <= s->cap; }

/* Field emission for one step: per patch, the field one spacing out along the
 * normal gives J, the expected number N = J A dt / e, and floor(N) electrons
 * plus one more with probability frac(N) are placed uniformly on the patch,
 * 10^-3 spacings outside the surface, with zero velocity. New ids are taken in
 * patch order. Returns the number injected, or -1 when capacity runs out. */
int64_t orc_fn_inject(const orc_config* c, uint32_t step, const double* phi, orc_species* e,
                      uint32_t* next_id, double* n_expected, int64_t* n_clamped) {
    int64_t np = orc_fn_patch_count(c), added = 0;
    double h = c->h;
    for (int64_t p = 0; p < np; ++p) {
        double g[8];
        orc_fn_patch(c, p, 0.5, 0.5, g);
        double F = orc_interp_phi(c, phi, g[0] + g[3], g[1] + g[4], g[2] + g[5]) / h;
        int cl = 0;
        double J = orc_fn_current(c, F, &cl);
        if (cl && n_clamped) *n_clamped += 1;
        double N = J * g[6] * h * h * c->dt / E_CH;
        if (n_expected) *n_expected += N;
        double u0, u1;
        draw2(c, (uint32_t)p, step, TAG_INJ, 0, &u0, &u1);
        double fl = floor(N);
        int64_t k = (int64_t)fl + ((u0 < N - fl) ? 1 : 0);
        if (!grow_ok(e, k)) return -1;
        for (int64_t j = 0; j < k; ++j) {
            double ua, ub;
            draw2(c, (uint32_t)p, step, TAG_INJ, (uint32_t)(1 + j), &ua, &ub);
            orc_fn_patch(c, p, ua, ub, g);
            int64_t m = e->n++;
            e->x[m] = g[0] + 1e-3 * g[3];
            e->y[m] = g[1] + 1e-3 * g[4];
            e->z[m] = g[2] + 1e-3 * g[5];
            e->vx[m] = e->vy[m] = e->vz[m] = 0.0;
            e->id[m] = (*next_id)++;
            if (e->w) e->w[m] = 1u;
            ++added;
        }
    }
    return added;
}

/* ------------------------------------------------------------------------ */
/* Neutral evaporation from the tip surface (Sec. 2.3.1): the Clausius-
 * Clapeyron flux
 *   phi_vap = p_atm / sqrt(2 pi m k_B T) exp[(E_vap / k_B)(1/T_b - 1/T)]
 * with p_atm = 101325 Pa, E_vap = 3.43 eV (the paper's value for Cu) and the
 * boiling point T_b of Cu, 2835 K (not printed in the paper), at a prescribed
 * uniform surface temperature T. Per emission patch N = phi_vap A dt atoms
 * are expected; floor(N) plus one more with probability frac(N) are placed
 * uniformly on the patch, 10^-3 spacings outside the surface. Reading of "speeds
 * sampled from the Maxwell-Boltzmann distribution based on the surface
 * temperature": the distribution of atoms leaving the surface at temperature
 * T, i.e. a Rayleigh-distributed normal component (flux weighting of the
 * Maxwellian) and Gaussian tangential components, each with variance
 * k_B T / m. Draws: (patch, step, EVAP, 0) for the count; for atom j,
 * (patch, step, EVAP, 1 + 3j) for the point, (.., 2 + 3j) and (.., 3 + 3j)
 * for the velocity. Returns the number added, or -1 when capacity runs out. */
#define TAG_EVAP 7u
#define P_ATM 101325.0
#define E_VAP_CU 3.43
#define T_BOIL_CU 2835.0
#define K_B 1.380649e-23

double orc_evap_flux(const orc_config* c, double T) {
    if (!(T > 0.0)) return 0.0;
    return P_ATM / sqrt(2.0 * PI * c->m_ion * K_B * T) * exp(E_VAP_CU * E_CH / K_B * (1.0 / T_BOIL_CU - 1.0 / T));
}

/* Weight of the superparticles injected at one surface location (Sec. 2.3.2):
 * w = min(ceil(max(1, sqrt((n_cell / n_max)(N_inj / w_min)))) w_min, w_max)
 * with w_min = 1, N_inj the atoms injected there in the step and n_cell the
 * superparticle number density of the cell above the location (reading: the
 * cell of the field point one spacing out along the normal, counted at the
 * last binning of the particles, i.e. after the last push). */
static int64_t inject_weight(const orc_config* c, int64_t n_inj, int64_t cell_sp) {
    if (c->w_max <= 1 || n_inj <= 1) return 1;
    double n_cell = (double)cell_sp / (c->h * c->h * c->h);
    double r = sqrt(n_cell / c->n_max * (double)n_inj);
    double w = ceil(r > 1.0 ? r : 1.0);
    return w < (double)c->w_max ? (int64_t)w : (int64_t)c->w_max;
}

int64_t orc_evaporate(const orc_config* c, uint32_t step, double T, orc_species* nsp, uint32_t* next_id,
                      double* n_expected, const int64_t* cell_count) {
    int64_t np = orc_fn_patch_count(c), added = 0;
    double h = c->h, flux = orc_evap_flux(c, T);
    double sig = sqrt(K_B * T / c->m_ion) * c->dt / h;   /* grid units per step */
    for (int64_t p = 0; p < np; ++p) {
        double g[8];
        orc_fn_patch(c, p, 0.5, 0.5, g);
        double N = flux * g[6] * h * h * c->dt;
        if (n_expected) *n_expected += N;
        double u0, u1;
        draw2(c, (uint32_t)p, step, TAG_EVAP, 0, &u0, &u1);
        double fl = floor(N);
        int64_t atoms = (int64_t)fl + ((u0 < N - fl) ? 1 : 0);
        /* atoms -> superparticles of weight wp (the last one takes the rest) */
        int64_t cnt = cell_count ? cell_count[orc_cell_of(c, g[0] + g[3], g[1] + g[4], g[2] + g[5])] : 0;
        int64_t wp = inject_weight(c, atoms, cnt);
        int64_t k = (atoms + wp - 1) / wp;
        if (!grow_ok(nsp, k)) return -1;
        for (int64_t j = 0; j < k; ++j) {
            double ua, ub, w1, w2, w3, unused;
            draw2(c, (uint32_t)p, step, TAG_EVAP, (uint32_t)(1 + 3 * j), &ua, &ub);
            draw2(c, (uint32_t)p, step, TAG_EVAP, (uint32_t)(2 + 3 * j), &w1, &w2);
            draw2(c, (uint32_t)p, step, TAG_EVAP, (uint32_t)(3 + 3 * j), &w3, &unused);
            orc_fn_patch(c, p, ua, ub, g);
            double n[3] = {g[3], g[4], g[5]};
            double tl = sqrt(n[0] * n[0] + n[1] * n[1]);
            double t1[3] = {-n[1] / tl, n[0] / tl, 0.0};
            double t2[3] = {n[1] * t1[2] - n[2] * t1[1], n[2] * t1[0] - n[0] * t1[2], n[0] * t1[1] - n[1] * t1[0]};
            double vn = sig * sqrt(-2.0 * log(w1));
            double rt = sig * sqrt(-2.0 * log(w2));
            double va = rt * cos(2.0 * PI * w3), vb = rt * sin(2.0 * PI * w3);
            int64_t m = nsp->n++;
            nsp->x[m] = g[0] + 1e-3 * n[0];
            nsp->y[m] = g[1] + 1e-3 * n[1];
            nsp->z[m] = g[2] + 1e-3 * n[2];
            nsp->vx[m] = vn * n[0] + va * t1[0] + vb * t2[0];
            nsp->vy[m] = vn * n[1] + va * t1[1] + vb * t2[1];
            nsp->vz[m] = vn * n[2] + va * t1[2] + vb * t2[2];
            nsp->id[m] = (*next_id)++;
            if (nsp->w) nsp->w[m] = (uint32_t)(j + 1 < k ? wp : atoms - (k - 1) * wp);
            ++added;
        }
    }
    return added;
}

/* ------------------------------------------------------------------------ */
/* Monte Carlo collisions (Sec. 2.2, Eqs. colp, du, newv; Table colls) and
 * direct field ionization (Sec. 2.3.4, Eq. dfi). */

typedef struct entry { int64_t cell; int32_t sp; uint32_t id; int64_t idx; } entry;

static int entry_cmp(const void* a, const void* b) {
    const entry* x = a; const entry* y = b;
    if (x->cell != y->cell) return x->cell < y->cell ? -1 : 1;
    if (x->sp != y->sp) return x->sp < y->sp ? -1 : 1;
    if (x->id != y->id) return x->id < y->id ? -1 : 1;
    return 0;
}

typedef struct product { int32_t kind; uint32_t nid; int64_t nidx; int64_t ev; double ve[3]; uint32_t c; } product;

/* A superparticle split off by a partial collision (Sec. 2.3.2): c of the
 * parent's weight units leave with the velocity v; the parent keeps the rest
 * and its velocity. Ordered by (species, parent id). */
typedef struct split { int32_t sp; uint32_t pid; int64_t pidx; double v[3]; uint32_t c; } split;

static int split_cmp(const void* a, const void* b) {
    const split* x = a; const split* y = b;
    if (x->sp != y->sp) return x->sp < y->sp ? -1 : 1;
    if (x->pid != y->pid) return x->pid < y->pid ? -1 : 1;
    return 0;
}

/* The c collided units of superparticle p of species s take velocity v: in
 * place when they are the whole superparticle, else split off. */
static void collided_units(orc_species* S, int s, int64_t p, const double v[3], uint32_t c, split* spl,
                           int64_t* nspl) {
    if (c >= wgt(S, p)) {
        S->vx[p] = v[0]; S->vy[p] = v[1]; S->vz[p] = v[2];
        return;
    }
    split* q = &spl[(*nspl)++];
    q->sp = s; q->pid = S->id[p]; q->pidx = p; q->c = c;
    q->v[0] = v[0]; q->v[1] = v[1]; q->v[2] = v[2];
}

static int product_cmp(const void* a, const void* b) {
    const product* x = a; const product* y = b;
    if (x->kind != y->kind) return x->kind < y->kind ? -1 : 1;
    if (x->nid != y->nid) return x->nid < y->nid ? -1 : 1;
    return 0;
}

static void isotropic(double ct, double ph, double s[3]) {
    double st = sqrt(1.0 - ct * ct);
    s[0] = st * cos(ph); s[1] = st * sin(ph); s[2] = ct;
}

static void fragile_add(orc_collide_out* o, uint32_t id) {
    if (o->n_fragile < o->fr_cap) o->fragile[o->n_fragile] = id;
    o->n_fragile++;
}

static int64_t event_add(orc_collide_out* o, int32_t kind, uint32_t a, uint32_t b) {
    if (o->n_ev < o->ev_cap) {
        orc_event* e = &o->ev[o->n_ev];
        e->kind = kind; e->id_a = a; e->id_b = b; e->new_ion = e->new_e = UINT32_MAX;
    }
    o->n_kind[kind]++;
    return o->n_ev++;
}

/* Elastic kick (Eqs. du, newv). u = v_A - v_B in SI; (theta, phi) are the
 * polar and azimuthal angles of u (the paper leaves them implicit; this is the
 * rotation that maps u onto the z axis), theta' and phi' the random isotropic
 * scattering angles. Returns the velocity difference Delta u. */
static void elastic_du(const double u[3], double ct2, double ph2, double du[3]) {
    double um = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    double up = sqrt(u[0] * u[0] + u[1] * u[1]);
    double ct = u[2] / um, st = up / um, cp = 1.0, sp = 0.0;
    if (up > 0.0) { cp = u[0] / up; sp = u[1] / up; }
    double st2 = sqrt(1.0 - ct2 * ct2);
    /* [R^{-1}(theta',phi') - I] (0,0,|u|)^T ; R^{-1} = R^T */
    double w0 = um * st2 * cos(ph2), w1 = um * st2 * sin(ph2), w2 = um * (ct2 - 1.0);
    /* R^{-1}(theta,phi) w */
    du[0] = ct * cp * w0 - sp * w1 + st * cp * w2;
    du[1] = ct * sp * w0 + cp * w1 + st * sp * w2;
    du[2] = -st * w0 + ct * w2;
}

/* One class of pair collisions in every cell. cls 1: (e, Cu) with elastic and
 * impact ionization; cls 2: (Cu+, Cu) with charge exchange.
 * Readings (the paper defers the pairing itself to its references):
 *  - the projectile species in a cell is the one with fewer particles (tie:
 *    the charged one); its particles, in ascending id order, take targets of
 *    the other species in ascending id order shifted cyclically by
 *    floor(U_c N_t) with U_c drawn per cell, so every target is hit at most
 *    once;
 *  - n is the target count over the full cell volume h^3 (weights are 1);
 *  - several processes of one class share one test with the summed cross
 *    section, P = 1 - exp(-u n sigma_tot dt) (Eq. colp), and a second uniform
 *    picks the process in proportion to its cross section;
 *  - the energy for sigma is (1/2) m_e u^2 for (e,Cu) and (1/2) m_Cu u^2 for
 *    (Cu+,Cu); ionization needs more than xi;
 *  - a particle takes part in at most one event per step: a neutral that had
 *    an (e,Cu) event is kept in the (Cu+,Cu) pairing but its pair is void.
 * Superparticle weights (Sec. 2.3.2, weights in units of w_min = 1): the
 * lighter superparticle of a pair is cut into N_p = min(w_a, w_b)
 * sub-particles of weight 1, each colliding with the heavier one (weight w_t)
 * with P = 1 - exp(-u n w_p w_t sigma dt), w_p = 1; N_coll counts the
 * sub-particles with U_i < P (U_0 is the pair's first draw, U_i for i >= 1
 * from the counter (projectile id, step, tag + 16, i)). The pair's event, its
 * process and its angles are drawn once; the N_coll collided units of each
 * side take the outcome, split off as a new superparticle where they are not
 * the whole of it (the rest keeps its velocity). With every weight 1 this is
 * the unweighted collision above. */
#define TAG_SUB 16u
static void mcc_class(const orc_config* c, uint32_t step, int cls, const entry* ent, int64_t ne,
                      orc_species* sp, uint8_t* used[3], product* prod, int64_t* nprod,
                      split* spl, int64_t* nspl, orc_collide_out* o) {
    int sa = (cls == 1) ? ORC_SP_E : ORC_SP_ION;
    int sb = ORC_SP_NEU;
    double ma = (cls == 1) ? M_EL : c->m_ion, mb = c->m_ion;
    double mu = ma * mb / (ma + mb);
    double h = c->h, dt = c->dt;
    double vol = h * h * h;
    int64_t s0 = 0;
    while (s0 < ne) {
        int64_t s1 = s0;
        while (s1 < ne && ent[s1].cell == ent[s0].cell) ++s1;
        /* ranges of species sa and sb inside [s0, s1), each sorted by id */
        int64_t a0 = s0, b0 = s0;
        while (a0 < s1 && ent[a0].sp != sa) ++a0;
        int64_t a1 = a0;
        while (a1 < s1 && ent[a1].sp == sa) ++a1;
        while (b0 < s1 && ent[b0].sp != sb) ++b0;
        int64_t b1 = b0;
        while (b1 < s1 && ent[b1].sp == sb) ++b1;
        int64_t NA = a1 - a0, NB = b1 - b0;
        if (NA > 0 && NB > 0) {
            int a_is_proj = NA <= NB;
            int64_t P0 = a_is_proj ? a0 : b0, NP = a_is_proj ? NA : NB;
            int64_t T0 = a_is_proj ? b0 : a0, NT = a_is_proj ? NB : NA;
            double uc, unused;
            draw2(c, (uint32_t)ent[s0].cell, step, cls == 1 ? TAG_PAIR1 : TAG_PAIR2, 0, &uc, &unused);
            int64_t shift = (int64_t)floor(uc * (double)NT);
            if (shift > NT - 1) shift = NT - 1;
            double n = (double)NT / vol;
            for (int64_t i = 0; i < NP; ++i) {
                const entry* pe = &ent[P0 + i];
                const entry* te = &ent[T0 + (shift + i) % NT];
                const entry* ea = a_is_proj ? pe : te;
                const entry* eb = a_is_proj ? te : pe;
                int64_t ia = ea->idx, ib = eb->idx;
                if (cls == 2 && used[sb][ib]) continue;
                orc_species* A = &sp[sa]; orc_species* B = &sp[sb];
                double u[3] = {(A->vx[ia] - B->vx[ib]) * h / dt, (A->vy[ia] - B->vy[ib]) * h / dt,
                               (A->vz[ia] - B->vz[ib]) * h / dt};
                double um = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                double E = 0.5 * (cls == 1 ? M_EL : c->m_ion) * um * um / E_CH;
                double sig[2];
                int nproc;
                if (cls == 1) {
                    sig[0] = orc_xs(c, c->xs_el, E);
                    sig[1] = (E > c->xi) ? orc_xs(c, c->xs_iz, E) : 0.0;
                    nproc = 2;
                } else {
                    sig[0] = orc_xs(c, c->xs_cx, E);
                    nproc = 1;
                }
                double stot = 0.0;
                for (int k = 0; k < nproc; ++k) stot += sig[k];
                uint32_t wa = wgt(A, ia), wb = wgt(B, ib);
                uint32_t wt = wa > wb ? wa : wb, npart = wa < wb ? wa : wb;
                double P = -expm1(-um * n * (double)wt * stot * dt);
                double U1, U2;
                draw2(c, pe->id, step, cls == 1 ? TAG_MCC1 : TAG_MCC2, 0, &U1, &U2);
                if (P > 0.0 && fabs(U1 - P) <= FRAGILE_REL * P) fragile_add(o, pe->id);
                uint32_t ncoll = (U1 < P) ? 1u : 0u;
                for (uint32_t q = 1; q < npart; ++q) {
                    double Uq, unq;
                    draw2(c, pe->id, step, (cls == 1 ? TAG_MCC1 : TAG_MCC2) + TAG_SUB, q, &Uq, &unq);
                    if (P > 0.0 && fabs(Uq - P) <= FRAGILE_REL * P) fragile_add(o, pe->id);
                    if (Uq < P) ++ncoll;
                }
                if (ncoll == 0) continue;
                int proc = nproc - 1;
                double cum = 0.0;
                for (int k = 0; k < nproc; ++k) {
                    cum += sig[k];
                    if (k < nproc - 1 && fabs(U2 * stot - cum) <= FRAGILE_REL * stot) fragile_add(o, pe->id);
                    if (U2 * stot < cum) { proc = k; break; }
                }
                used[sa][ia] = 1;
                used[sb][ib] = 1;
                if (cls == 1 && proc == 0) {
                    double u3, u4, du[3];
                    draw2(c, pe->id, step, TAG_MCC1, 1, &u3, &u4);
                    elastic_du(u, 2.0 * u3 - 1.0, 2.0 * PI * u4, du);
                    double ka = mu / ma * dt / h, kb = mu / mb * dt / h;
                    double va[3] = {A->vx[ia] + ka * du[0], A->vy[ia] + ka * du[1], A->vz[ia] + ka * du[2]};
                    double vb[3] = {B->vx[ib] - kb * du[0], B->vy[ib] - kb * du[1], B->vz[ib] - kb * du[2]};
                    collided_units(A, sa, ia, va, ncoll, spl, nspl);
                    collided_units(B, sb, ib, vb, ncoll, spl, nspl);
                    event_add(o, 1, A->id[ia], B->id[ib]);
                    o->n_kind_w[1] += ncoll;
                } else if (cls == 1) {
                    /* Impact ionization Cu + e -> Cu+ + 2e (Table colls). Reading
                     * (the paper defers details to its references): in the rest
                     * frame of the neutral the energy above xi is split as U5 and
                     * 1-U5 between the scattered and the new electron, each
                     * leaving isotropically; the ion keeps the neutral's position
                     * and velocity; the new electron starts at that position. */
                    double c1, p1, c2, p2, u5, unused2, s1v[3], s2v[3];
                    draw2(c, pe->id, step, TAG_MCC1, 1, &c1, &p1);
                    draw2(c, pe->id, step, TAG_MCC1, 2, &c2, &p2);
                    draw2(c, pe->id, step, TAG_MCC1, 3, &u5, &unused2);
                    isotropic(2.0 * c1 - 1.0, 2.0 * PI * p1, s1v);
                    isotropic(2.0 * c2 - 1.0, 2.0 * PI * p2, s2v);
                    double erem = E - c->xi;
                    double e1 = u5 * erem, e2 = erem - e1;
                    double w1 = sqrt(2.0 * e1 * E_CH / M_EL), w2 = sqrt(2.0 * e2 * E_CH / M_EL);
                    double vn[3] = {B->vx[ib] * h / dt, B->vy[ib] * h / dt, B->vz[ib] * h / dt};
                    double v1[3] = {(vn[0] + w1 * s1v[0]) * dt / h, (vn[1] + w1 * s1v[1]) * dt / h,
                                    (vn[2] + w1 * s1v[2]) * dt / h};
                    collided_units(A, sa, ia, v1, ncoll, spl, nspl);
                    product* pr = &prod[(*nprod)++];
                    pr->kind = 0; pr->nid = B->id[ib]; pr->nidx = ib; pr->c = ncoll;
                    pr->ve[0] = (vn[0] + w2 * s2v[0]) * dt / h;
                    pr->ve[1] = (vn[1] + w2 * s2v[1]) * dt / h;
                    pr->ve[2] = (vn[2] + w2 * s2v[2]) * dt / h;
                    pr->ev = event_add(o, 2, A->id[ia], B->id[ib]);
                    o->n_kind_w[2] += ncoll;
                } else {
                    /* Charge exchange Cu+ + Cu -> Cu + Cu+ (Table colls): the
                     * fast ion becomes a fast neutral and vice versa, i.e. the
                     * two velocities are exchanged while ids stay put. */
                    double va[3] = {B->vx[ib], B->vy[ib], B->vz[ib]};
                    double vb[3] = {A->vx[ia], A->vy[ia], A->vz[ia]};
                    collided_units(A, sa, ia, va, ncoll, spl, nspl);
                    collided_units(B, sb, ib, vb, ncoll, spl, nspl);
                    event_add(o, 3, A->id[ia], B->id[ib]);
                    o->n_kind_w[3] += ncoll;
                }
            }
        }
        s0 = s1;
    }
}

/* ------------------------------------------------------------------------ */
/* Same-species and Coulomb pairing (Table colls: elastic Cu + Cu, Coulomb
 * collisions between all charged particles). The paper names the processes
 * and cites Takizuka and Abe for the Coulomb collisions without restating
 * them; the readings here:
 *  - the particles of one species in a cell (those present before this
 *    step's collisions, unweighted), in ascending id order, are rotated
 *    cyclically by floor(U_c N) (U_c drawn per cell) and paired
 *    consecutively: (q0, q1), (q2, q3), ...;
 *  - Cu + Cu elastic: hard spheres of cross section sigma_nn, a pair
 *    collides when U1 < P = 1 - exp(-u n sigma_nn dt) with n = N / h^3, and
 *    scatters isotropically in its centre-of-mass frame (Eq. du with
 *    theta' = acos(2 U3 - 1), phi' = 2 pi U4); neutrals that had an event
 *    this step sit out, and with N odd the last one;
 *  - Coulomb (Takizuka-Abe): every pair scatters by theta = 2 atan(delta),
 *    delta normal with variance q_a^2 q_b^2 n_L ln(Lambda) dt /
 *    (8 pi eps0^2 mu^2 u^3), phi' uniform, applied through Eq. du; for the
 *    same species n_L = N / h^3, and with N odd the first three particles
 *    collide pairwise ((q0,q1), (q1,q2), (q2,q0)) with dt / 2 each; between
 *    electrons and ions the more numerous species' particles, in ascending id
 *    order, meet the other species' particles in ascending id order shifted
 *    cyclically by floor(U_c N_f) (so those are reused, one after another),
 *    with n_L the smaller density; a pair with u = 0 does not scatter. */
#define TAG_PAIR_NN 8u
#define TAG_NN 9u
#define TAG_PAIR_EE 10u
#define TAG_PAIR_II 11u
#define TAG_PAIR_EI 12u
#define TAG_COUL 13u
#define TAG_COUL_EI 14u

/* One Takizuka-Abe scattering of a (species sa, index ia) with (sb, ib) over
 * a time dts at the density n_l; draws keyed by (subject, step, tag). */
static int ta_scatter(const orc_config* c, uint32_t step, uint32_t subject, uint32_t tag, orc_species* A, int sa,
                      int64_t ia, orc_species* B, int sb, int64_t ib, double n_l, double dts) {
    double h = c->h, dt = c->dt;
    double ma = (sa == ORC_SP_E) ? M_EL : c->m_ion, mb = (sb == ORC_SP_E) ? M_EL : c->m_ion;
    double qa = (sa == ORC_SP_E) ? -E_CH : E_CH, qb = (sb == ORC_SP_E) ? -E_CH : E_CH;
    double mu = ma * mb / (ma + mb);
    double u[3] = {(A->vx[ia] - B->vx[ib]) * h / dt, (A->vy[ia] - B->vy[ib]) * h / dt,
                   (A->vz[ia] - B->vz[ib]) * h / dt};
    double um = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    if (!(um > 0.0)) return 0;
    double var = qa * qa * qb * qb * n_l * c->coulomb_log * dts / (8.0 * PI * EPS0 * EPS0 * mu * mu * um * um * um);
    double u1, u2, u3, unused;
    draw2(c, subject, step, tag, 0, &u1, &u2);
    draw2(c, subject, step, tag, 1, &u3, &unused);
    double delta = sqrt(var) * sqrt(-2.0 * log(u1)) * cos(2.0 * PI * u2);
    double ct = (1.0 - delta * delta) / (1.0 + delta * delta);
    double du[3];
    elastic_du(u, ct, 2.0 * PI * u3, du);
    double ka = mu / ma * dt / h, kb = mu / mb * dt / h;
    A->vx[ia] += ka * du[0]; A->vy[ia] += ka * du[1]; A->vz[ia] += ka * du[2];
    B->vx[ib] -= kb * du[0]; B->vy[ib] -= kb * du[1]; B->vz[ib] -= kb * du[2];
    return 1;
}

/* kind 0: Cu-Cu elastic; 1: e-e Coulomb; 2: Cu+-Cu+ Coulomb. Returns the
 * number of collisions (kind 0) or scatterings. */
static int64_t pair_same(const orc_config* c, uint32_t step, int kind, const entry* ent, int64_t ne, orc_species* sp,
                         uint8_t* used[3]) {
    int64_t count = 0;
    int s = kind == 0 ? ORC_SP_NEU : (kind == 1 ? ORC_SP_E : ORC_SP_ION);
    uint32_t tpair = kind == 0 ? TAG_PAIR_NN : (kind == 1 ? TAG_PAIR_EE : TAG_PAIR_II);
    orc_species* S = &sp[s];
    double vol = c->h * c->h * c->h, h = c->h, dt = c->dt;
    int64_t* q = malloc((ne + 1) * sizeof(int64_t));
    int64_t s0 = 0;
    while (s0 < ne) {
        int64_t s1 = s0;
        while (s1 < ne && ent[s1].cell == ent[s0].cell) ++s1;
        int64_t a0 = s0;
        while (a0 < s1 && ent[a0].sp != s) ++a0;
        int64_t a1 = a0;
        while (a1 < s1 && ent[a1].sp == s) ++a1;
        int64_t N = a1 - a0;
        if (N >= 2) {
            double uc, unused;
            draw2(c, (uint32_t)ent[s0].cell, step, tpair, 0, &uc, &unused);
            int64_t shift = (int64_t)floor(uc * (double)N);
            if (shift > N - 1) shift = N - 1;
            for (int64_t j = 0; j < N; ++j) q[j] = ent[a0 + (shift + j) % N].idx;
            double n = (double)N / vol;
            if (kind == 0) {
                for (int64_t j = 0; j + 1 < N; j += 2) {
                    int64_t ia = q[j], ib = q[j + 1];
                    if (used[s][ia] || used[s][ib]) continue;
                    double u[3] = {(S->vx[ia] - S->vx[ib]) * h / dt, (S->vy[ia] - S->vy[ib]) * h / dt,
                                   (S->vz[ia] - S->vz[ib]) * h / dt};
                    double um = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                    double P = -expm1(-um * n * c->sigma_nn * dt);
                    double U1, unused2, u3, u4;
                    draw2(c, S->id[ia], step, TAG_NN, 0, &U1, &unused2);
                    if (!(U1 < P)) continue;
                    draw2(c, S->id[ia], step, TAG_NN, 1, &u3, &u4);
                    double du[3];
                    elastic_du(u, 2.0 * u3 - 1.0, 2.0 * PI * u4, du);
                    double k = 0.5 * dt / h;   /* mu / m = 1/2 */
                    S->vx[ia] += k * du[0]; S->vy[ia] += k * du[1]; S->vz[ia] += k * du[2];
                    S->vx[ib] -= k * du[0]; S->vy[ib] -= k * du[1]; S->vz[ib] -= k * du[2];
                    ++count;
                }
            } else {
                int64_t j0 = 0;
                if (N % 2 == 1) {
                    /* the first three pairwise with half the time step */
                    count += ta_scatter(c, step, S->id[q[0]], TAG_COUL, S, s, q[0], S, s, q[1], n, 0.5 * dt);
                    count += ta_scatter(c, step, S->id[q[1]], TAG_COUL, S, s, q[1], S, s, q[2], n, 0.5 * dt);
                    count += ta_scatter(c, step, S->id[q[2]], TAG_COUL, S, s, q[2], S, s, q[0], n, 0.5 * dt);
                    j0 = 3;
                }
                for (int64_t j = j0; j + 1 < N; j += 2)
                    count += ta_scatter(c, step, S->id[q[j]], TAG_COUL, S, s, q[j], S, s, q[j + 1], n, dt);
            }
        }
        s0 = s1;
    }
    free(q);
    return count;
}

static int64_t coulomb_e_ion(const orc_config* c, uint32_t step, const entry* ent, int64_t ne, orc_species* sp) {
    int64_t count = 0;
    double vol = c->h * c->h * c->h, dt = c->dt;
    int64_t s0 = 0;
    while (s0 < ne) {
        int64_t s1 = s0;
        while (s1 < ne && ent[s1].cell == ent[s0].cell) ++s1;
        int64_t e0 = s0;
        while (e0 < s1 && ent[e0].sp != ORC_SP_E) ++e0;
        int64_t e1 = e0;
        while (e1 < s1 && ent[e1].sp == ORC_SP_E) ++e1;
        int64_t i0 = s0;
        while (i0 < s1 && ent[i0].sp != ORC_SP_ION) ++i0;
        int64_t i1 = i0;
        while (i1 < s1 && ent[i1].sp == ORC_SP_ION) ++i1;
        int64_t NE = e1 - e0, NI = i1 - i0;
        if (NE > 0 && NI > 0) {
            /* the more numerous species meets the other (tie: electrons meet ions) */
            int e_more = NE >= NI;
            int64_t M0 = e_more ? e0 : i0, NM = e_more ? NE : NI;
            int64_t F0 = e_more ? i0 : e0, NF = e_more ? NI : NE;
            double uc, unused;
            draw2(c, (uint32_t)ent[s0].cell, step, TAG_PAIR_EI, 0, &uc, &unused);
            int64_t shift = (int64_t)floor(uc * (double)NF);
            if (shift > NF - 1) shift = NF - 1;
            double n_l = (double)NF / vol;
            for (int64_t i = 0; i < NM; ++i) {
                const entry* m = &ent[M0 + i];
                const entry* f = &ent[F0 + (shift + i) % NF];
                const entry* ee = e_more ? m : f;
                const entry* ei = e_more ? f : m;
                count += ta_scatter(c, step, m->id, TAG_COUL_EI, &sp[ORC_SP_E], ORC_SP_E, ee->idx, &sp[ORC_SP_ION],
                                    ORC_SP_ION, ei->idx, n_l, dt);
            }
        }
        s0 = s1;
    }
    return count;
}

/* Recombination Cu+ + e -> Cu (Table colls; the cited cross sections are not
 * given, so a constant sigma_rec stands in). Readings: electrons and ions of
 * a cell (present before this step's collisions) are paired like the
 * collision classes above -- the fewer species (tie: the ions) as
 * projectiles in ascending id order, targets in ascending id order shifted
 * by floor(U_c N_t) -- and a pair recombines when U1 < P = 1 - exp(-u n
 * sigma_rec dt), n = N_t / h^3; earlier events of the step do not exclude a
 * particle. The atom takes the ion's position and the pair's centre-of-mass
 * velocity (momentum conserved; the binding energy and the kinetic energy of
 * the relative motion leave the system). */
#define TAG_PAIR_REC 32u
#define TAG_REC 33u

typedef struct recomb { uint32_t ion_id; int64_t iidx, eidx; double v[3]; } recomb;

static int recomb_cmp(const void* a, const void* b) {
    const recomb* x = a; const recomb* y = b;
    return x->ion_id < y->ion_id ? -1 : (x->ion_id > y->ion_id ? 1 : 0);
}

static int64_t recombine(const orc_config* c, uint32_t step, const entry* ent, int64_t ne, orc_species* sp,
                         recomb* rec) {
    double vol = c->h * c->h * c->h, h = c->h, dt = c->dt;
    orc_species* El = &sp[ORC_SP_E]; orc_species* I = &sp[ORC_SP_ION];
    int64_t nrec = 0, s0 = 0;
    while (s0 < ne) {
        int64_t s1 = s0;
        while (s1 < ne && ent[s1].cell == ent[s0].cell) ++s1;
        int64_t e0 = s0;
        while (e0 < s1 && ent[e0].sp != ORC_SP_E) ++e0;
        int64_t e1 = e0;
        while (e1 < s1 && ent[e1].sp == ORC_SP_E) ++e1;
        int64_t i0 = s0;
        while (i0 < s1 && ent[i0].sp != ORC_SP_ION) ++i0;
        int64_t i1 = i0;
        while (i1 < s1 && ent[i1].sp == ORC_SP_ION) ++i1;
        int64_t NE = e1 - e0, NI = i1 - i0;
        if (NE > 0 && NI > 0) {
            int ion_proj = NI <= NE;
            int64_t P0 = ion_proj ? i0 : e0, NP = ion_proj ? NI : NE;
            int64_t T0 = ion_proj ? e0 : i0, NT = ion_proj ? NE : NI;
            double uc, unused;
            draw2(c, (uint32_t)ent[s0].cell, step, TAG_PAIR_REC, 0, &uc, &unused);
            int64_t rs = (int64_t)floor(uc * (double)NT);
            if (rs > NT - 1) rs = NT - 1;
            double n = (double)NT / vol;
            for (int64_t i = 0; i < NP; ++i) {
                const entry* pj = &ent[P0 + i];
                const entry* tg = &ent[T0 + (rs + i) % NT];
                int64_t ii = ion_proj ? pj->idx : tg->idx, ie = ion_proj ? tg->idx : pj->idx;
                double u[3] = {(El->vx[ie] - I->vx[ii]) * h / dt, (El->vy[ie] - I->vy[ii]) * h / dt,
                               (El->vz[ie] - I->vz[ii]) * h / dt};
                double um = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                double P = -expm1(-um * n * c->sigma_rec * dt);
                double U1, unused2;
                draw2(c, pj->id, step, TAG_REC, 0, &U1, &unused2);
                if (!(U1 < P)) continue;
                recomb* r = &rec[nrec++];
                r->ion_id = I->id[ii]; r->iidx = ii; r->eidx = ie;
                double mt = M_EL + c->m_ion;
                r->v[0] = (M_EL * El->vx[ie] + c->m_ion * I->vx[ii]) / mt;
                r->v[1] = (M_EL * El->vy[ie] + c->m_ion * I->vy[ii]) / mt;
                r->v[2] = (M_EL * El->vz[ie] + c->m_ion * I->vz[ii]) / mt;
            }
        }
        s0 = s1;
    }
    return nrec;
}

/* Collisions of one step on the post-push state: (e,Cu) pairs, then (Cu+,Cu)
 * pairs, then field ionization of every neutral without an event, then (with
 * their flags) Cu-Cu elastic pairs, e-e, Cu+-Cu+ and e-Cu+ Coulomb pairs and
 * recombination, then the products. Ionization products (impact and field) are created in the order
 * (impact before field, ascending neutral id), each taking two new ids: the ion
 * first, then the electron; each carries the N_coll ionized units, which the
 * neutral loses. Then the split-off superparticles, in the order (species,
 * parent id), each taking one new id. Neutrals left without weight are
 * removed (order preserved). */
int orc_collide(const orc_config* c, uint32_t step, int32_t flags, const double* E,
                orc_species* sp, uint32_t* next_id, orc_collide_out* o) {
    int64_t ne = sp[0].n + sp[1].n + sp[2].n;
    entry* ent = malloc((ne + 1) * sizeof(entry));
    int64_t m = 0;
    for (int s = 0; s < 3; ++s)
        for (int64_t p = 0; p < sp[s].n; ++p) {
            ent[m].cell = orc_cell_of(c, sp[s].x[p], sp[s].y[p], sp[s].z[p]);
            ent[m].sp = s; ent[m].id = sp[s].id[p]; ent[m].idx = p; ++m;
        }
    qsort(ent, ne, sizeof(entry), entry_cmp);
    uint8_t* used[3];
    for (int s = 0; s < 3; ++s) used[s] = calloc(sp[s].n + 1, 1);
    product* prod = malloc((sp[2].n + 1) * sizeof(product));
    int64_t nprod = 0;
    split* spl = malloc((ne + 1) * sizeof(split));
    int64_t nspl = 0;
    o->n_ev = 0; o->n_fragile = 0; o->n_bsi_skip = 0; o->n_split = 0;
    for (int k = 0; k < 5; ++k) { o->n_kind[k] = 0; o->n_kind_w[k] = 0; }

    if (flags & ORC_COLL_MCC1) mcc_class(c, step, 1, ent, ne, sp, used, prod, &nprod, spl, &nspl, o);
    if (flags & ORC_COLL_MCC2) mcc_class(c, step, 2, ent, ne, sp, used, prod, &nprod, spl, &nspl, o);

    if (flags & ORC_COLL_FI) {
        /* Field ionization (Sec. 2.3.4): a neutral ionizes in the step when
         * P dt > U, P from Eq. dfi at the local field. Readings: the field is
         * taken at the post-push position; the paper leaves neutrals in
         * fields above the barrier-suppression limit E > (3/2) xi^{3/2} out of
         * the rate, read as: no field ionization is attempted for them; the
         * products are placed as in impact ionization, the electron with the
         * neutral's velocity. */
        orc_species* N = &sp[ORC_SP_NEU];
        double ebsi = 1.5 * pow(c->xi, 1.5);
        double dt_fs = c->dt * 1e15;
        for (int64_t p = 0; p < N->n; ++p) {
            double e[3];
            orc_gather(c, E, N->x[p], N->y[p], N->z[p], e);
            double Eg = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]) * 1e-9;
            if (Eg > ebsi) { o->n_bsi_skip++; continue; }  /* counted for every neutral */
            if (used[ORC_SP_NEU][p]) continue;
            double pdt = orc_adk_rate(c, Eg) * dt_fs;
            double U, unused;
            draw2(c, N->id[p], step, TAG_FI, 0, &U, &unused);
            if (pdt > 0.0 && fabs(U - pdt) <= FRAGILE_FI * pdt) fragile_add(o, N->id[p]);
            /* a neutral superparticle of weight w: each of its w units ionizes
             * when P dt > U_i (U_0 above, U_i from (id, step, FI + 16, i)) */
            uint32_t ncoll = (pdt > U) ? 1u : 0u;
            for (uint32_t q = 1; q < wgt(N, p); ++q) {
                double Uq, unq;
                draw2(c, N->id[p], step, TAG_FI + TAG_SUB, q, &Uq, &unq);
                if (pdt > 0.0 && fabs(Uq - pdt) <= FRAGILE_FI * pdt) fragile_add(o, N->id[p]);
                if (pdt > Uq) ++ncoll;
            }
            if (ncoll > 0) {
                used[ORC_SP_NEU][p] = 1;
                product* pr = &prod[nprod++];
                pr->kind = 1; pr->nid = N->id[p]; pr->nidx = p; pr->c = ncoll;
                pr->ve[0] = N->vx[p]; pr->ve[1] = N->vy[p]; pr->ve[2] = N->vz[p];
                pr->ev = event_add(o, 4, UINT32_MAX, N->id[p]);
                o->n_kind_w[4] += ncoll;
            }
        }
    }

    o->n_nn = 0; o->n_coul = 0;
    if (flags & ORC_COLL_NN) o->n_nn = pair_same(c, step, 0, ent, ne, sp, used);
    if (flags & ORC_COLL_COUL) {
        o->n_coul += pair_same(c, step, 1, ent, ne, sp, used);
        o->n_coul += pair_same(c, step, 2, ent, ne, sp, used);
        o->n_coul += coulomb_e_ion(c, step, ent, ne, sp);
    }
    recomb* rec = malloc((ne + 1) * sizeof(recomb));
    int64_t nrec = (flags & ORC_COLL_REC) ? recombine(c, step, ent, ne, sp, rec) : 0;
    qsort(rec, nrec, sizeof(recomb), recomb_cmp);
    o->n_rec = nrec;

    int rc = 0;
    qsort(prod, nprod, sizeof(product), product_cmp);
    qsort(spl, nspl, sizeof(split), split_cmp);
    orc_species* I = &sp[ORC_SP_ION]; orc_species* El = &sp[ORC_SP_E]; orc_species* N = &sp[ORC_SP_NEU];
    int64_t nsp_new[3] = {0, 0, 0};
    for (int64_t k = 0; k < nspl; ++k) nsp_new[spl[k].sp]++;
    if (!grow_ok(I, nprod + nsp_new[ORC_SP_ION]) || !grow_ok(El, nprod + nsp_new[ORC_SP_E]) ||
        !grow_ok(N, nsp_new[ORC_SP_NEU] + nrec))
        rc = -1;
    uint8_t* dead = calloc(N->n + nsp_new[ORC_SP_NEU] + nrec + 1, 1);
    for (int64_t k = 0; k < nprod && rc == 0; ++k) {
        product* pr = &prod[k];
        int64_t ni = pr->nidx;
        uint32_t id_ion = (*next_id)++, id_e = (*next_id)++;
        int64_t a = I->n++;
        I->x[a] = N->x[ni]; I->y[a] = N->y[ni]; I->z[a] = N->z[ni];
        I->vx[a] = N->vx[ni]; I->vy[a] = N->vy[ni]; I->vz[a] = N->vz[ni];
        I->id[a] = id_ion;
        if (I->w) I->w[a] = pr->c;
        int64_t b = El->n++;
        El->x[b] = N->x[ni]; El->y[b] = N->y[ni]; El->z[b] = N->z[ni];
        El->vx[b] = pr->ve[0]; El->vy[b] = pr->ve[1]; El->vz[b] = pr->ve[2];
        El->id[b] = id_e;
        if (El->w) El->w[b] = pr->c;
        if (N->w && N->w[ni] > pr->c) N->w[ni] -= pr->c;
        else dead[ni] = 1;
        if (pr->ev < o->ev_cap) { o->ev[pr->ev].new_ion = id_ion; o->ev[pr->ev].new_e = id_e; }
    }
    /* split-off superparticles at their parents' positions */
    for (int64_t k = 0; k < nspl && rc == 0; ++k) {
        split* q = &spl[k];
        orc_species* S = &sp[q->sp];
        int64_t a = S->n++;
        S->x[a] = S->x[q->pidx]; S->y[a] = S->y[q->pidx]; S->z[a] = S->z[q->pidx];
        S->vx[a] = q->v[0]; S->vy[a] = q->v[1]; S->vz[a] = q->v[2];
        S->id[a] = (*next_id)++;
        S->w[a] = q->c;
        S->w[q->pidx] -= q->c;
    }
    o->n_split = nspl;
    /* recombination products in ascending ion id, after the other products;
     * the electron and the ion are removed */
    uint8_t* dead_e = calloc(El->n + 1, 1);
    uint8_t* dead_i = calloc(I->n + 1, 1);
    for (int64_t k = 0; k < nrec && rc == 0; ++k) {
        recomb* r = &rec[k];
        int64_t a = N->n++;
        N->x[a] = I->x[r->iidx]; N->y[a] = I->y[r->iidx]; N->z[a] = I->z[r->iidx];
        N->vx[a] = r->v[0]; N->vy[a] = r->v[1]; N->vz[a] = r->v[2];
        N->id[a] = (*next_id)++;
        if (N->w) N->w[a] = 1;
        dead_e[r->eidx] = 1;
        dead_i[r->iidx] = 1;
    }
    for (int pass = 0; pass < 2 && nrec > 0; ++pass) {
        orc_species* S = pass == 0 ? El : I;
        uint8_t* dd = pass == 0 ? dead_e : dead_i;
        int64_t w = 0;
        for (int64_t p = 0; p < S->n; ++p) {
            if (dd[p]) continue;
            S->x[w] = S->x[p]; S->y[w] = S->y[p]; S->z[w] = S->z[p];
            S->vx[w] = S->vx[p]; S->vy[w] = S->vy[p]; S->vz[w] = S->vz[p];
            S->id[w] = S->id[p];
            if (S->w) S->w[w] = S->w[p];
            ++w;
        }
        S->n = w;
    }
    free(dead_e); free(dead_i); free(rec);
    /* remove the neutrals left without weight, keeping the order of the others */
    int64_t w = 0;
    for (int64_t p = 0; p < N->n; ++p) {
        if (dead[p]) continue;
        N->x[w] = N->x[p]; N->y[w] = N->y[p]; N->z[w] = N->z[p];
        N->vx[w] = N->vx[p]; N->vy[w] = N->vy[p]; N->vz[w] = N->vz[p];
        N->id[w] = N->id[p];
        if (N->w) N->w[w] = N->w[p];
        ++w;
    }
    N->n = w;
    free(dead); free(prod); free(spl); free(ent);
    for (int s = 0; s < 3; ++s) free(used[s]);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Moments: kinetic energy per species [J], the Shockley-Ramo gap current
 * I = sum w q v . E0(r) [A] (w the superparticle weight) with E0 the field of the unit-anode Laplace problem
 * (Sec. 2.3.1), evaluated on the stored state (positions x^{n+1}, velocities
 * v^{n+1/2}), and the particle counts. out = {KE_e, KE_ion, KE_neu, I_SR,
 * n_e, n_ion, n_neu, 0}. */
void orc_moments(const orc_config* c, const orc_species* sp, const double* E0, double out[8]) {
    double mass[3] = {M_EL, c->m_ion, c->m_ion};
    double charge[3] = {-E_CH, E_CH, 0.0};
    double sv = c->h / c->dt;
    double isr = 0.0;
    for (int s = 0; s < 3; ++s) {
        double ke = 0.0;
        for (int64_t p = 0; p < sp[s].n; ++p) {
            double vx = sp[s].vx[p] * sv, vy = sp[s].vy[p] * sv, vz = sp[s].vz[p] * sv;
            double wp = (double)wgt(&sp[s], p);
            ke += wp * 0.5 * mass[s] * (vx * vx + vy * vy + vz * vz);
            if (charge[s] != 0.0) {
                double e[3];
                orc_gather(c, E0, sp[s].x[p], sp[s].y[p], sp[s].z[p], e);
                isr += wp * charge[s] * (vx * e[0] + vy * e[1] + vz * e[2]);
            }
        }
        out[s] = ke;
        out[4 + s] = (double)sp[s].n;
    }
    out[3] = isr;
    out[7] = 0.0;
}
