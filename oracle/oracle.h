/*
 * oracle.h -- plain FP64 CPU oracle of the two-component Shan-Chen D3Q19
 * lattice Boltzmann step with interacting walls, and of the contact-angle
 * observable measured on it.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against the paper.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never does.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Sources (Schmieschek & Harting, "Contact angle determination in
 * multicomponent lattice Boltzmann simulations"):
 *   Sec. 2, Eq. (LBeqs)      multi-species stream + collide update
 *   Sec. 2, BGK operator     single relaxation time per species
 *   Sec. 2, Eq. (Equil)      third-order equilibrium, D3Q19 lattice
 *   Sec. 2, Eq. (SCforce)    Shan-Chen mean-field force, nearest neighbours
 *   Sec. 2, velocity shift   du = tau F / rho added to u in the equilibrium
 *   Sec. 2, wall model       mid-grid bounce-back; wall nodes act as an
 *                            extra species with constant rest density
 *   Sec. 2, order parameter  phi = rho_A - rho_B, interface at phi = 0
 *   Sec. 3, Eq. (geoCA)      geometric contact angle from base and height
 *                            measured relative to a reference plane 5 l.u.
 *                            above the wall
 * The adjoint (reverse-mode derivative of the step) is an extension that the
 * paper does not contain; it is the exact transpose of each forward sub-step.
 *
 * Layout (the oracle's own, unlike the GPU library): array-of-structures,
 * f[((z*ny + y)*nx + x)*38 + a*19 + k], x fastest, species a in {0=A, 1=B}.
 * Density / scalar fields: s[((z*ny + y)*nx + x)*2 + a].
 * All axes wrap periodically; walls come only from the solid mask.
 */
#ifndef SC_ORACLE_H
#define SC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORA_Q 19

typedef struct {
  int32_t nx, ny, nz;
  int32_t psi;          /* 0: psi(rho) = rho ; 1: psi(rho) = 1 - exp(-rho) */
  double tau[2];        /* relaxation times of A and B, > 1/2 */
  double g_ab;          /* fluid-fluid coupling, > 0 repulsive */
  double g_wall[2];     /* coupling felt by A and by B from wall nodes */
  double rho_wall[2];   /* wall pseudo-density: A-content and B-content */
  double w_axis, w_diag;/* per-direction weights of the force sum (1, 1) */
} ora_params;

typedef struct {
  int32_t ic, jc;       /* column of the droplet axis */
  int32_t z_solid_top;  /* top solid layer under the droplet */
  int32_t offset;       /* reference layer = z_solid_top + offset */
  double eps;           /* half width of the smoothed indicator (E2) */
} ora_ca_cfg;

/* result of the contact-angle observable; angles in degrees */
typedef struct {
  double theta_e1, h_e1, a_e1, R_e1, aref_e1, H_e1;
  double theta_e2, h_e2, a_e2, R_e2, aref_e2, H_e2;
  double cx, cy;        /* centroid of phi > 0 in the reference layer */
  int32_t flags;
  int32_t pad;
} ora_ca;

/* flags of ora_ca */
#define ORA_CA_NO_REF     1   /* phi <= 0 at the reference layer: direct fallback */
#define ORA_CA_E1_FLAT    2   /* E1: a^2 <= 0, angle reported as 180 deg */
#define ORA_CA_E2_FLAT    4   /* E2: a^2 <= 0, angle reported as 180 deg */
#define ORA_CA_RAY_LIMIT  8   /* a half-chord ray found no crossing within L/2 */
#define ORA_CA_NO_APEX   16   /* no phi crossing above the reference layer */
#define ORA_CA_NO_DROP   32   /* no droplet on the column: angle is NaN */
#define ORA_CA_E2_EMPTY  64   /* E2 column height H <= 0 */
#define ORA_CA_E2_WHOLE_LAYER 128 /* E2 summed the whole reference layer */

typedef struct ora_lattice ora_lattice;

/* lattice tables: velocities c[19][3], weights w[19], opposite index opp[19] */
void ora_tables(int32_t* c, double* w, int32_t* opp);

/* third-order equilibrium of one species (Eq. Equil), out[19] */
void ora_equilibrium(double rho, const double* u, double* out);

ora_lattice* ora_create(const ora_params* p, const uint8_t* solid);
void ora_destroy(ora_lattice* L);
int ora_set_params(ora_lattice* L, const ora_params* p);

/* C_k = zeta_k rho (u = 0) at fluid nodes; rho_a, rho_b are nx*ny*nz fields */
void ora_init_equilibrium(ora_lattice* L, const double* rho_a, const double* rho_b);
/* C_k = n^eq_k(rho, u) with the same velocity u (3 per node) for both species */
void ora_init_equilibrium_u(ora_lattice* L, const double* rho_a, const double* rho_b,
                            const double* u);

void ora_step(ora_lattice* L, int64_t nsteps);
int64_t ora_step_count(const ora_lattice* L);

void ora_get_state(const ora_lattice* L, double* dst);
void ora_set_state(ora_lattice* L, const double* src);

/* rho[node*2 + a] = sum_k C_k^a at fluid nodes, 0 at solid nodes */
void ora_density(const ora_lattice* L, double* rho);
/* out = {mass_A, mass_B, P_x, P_y, P_z, finite(0/1)} */
void ora_observables(const ora_lattice* L, double* out);

/* The sub-steps of one step, exposed so that tests can check each one. */
/* streaming with mid-grid bounce-back applied to an arbitrary field 'in' */
void ora_stream(const ora_lattice* L, const double* in, double* out);
/* Shan-Chen + wall force from post-stream densities rho (2 per node):
   F[node*6 + a*3 + d] */
void ora_force(const ora_lattice* L, const double* rho, double* F);

/* Pressure tensor (Sec. 4.1) of the current state at every node:
   P[node*6 + {xx, yy, zz, xy, xz, yz}]; at solid nodes the wall's half of
   the wall-fluid pair terms (no kinetic part). */
void ora_pressure_tensor(ora_lattice* L, double* P);
/* Surface tension integral (Eq. gammaMechDef) for interfaces normal to z:
   sum over planes of the plane mean (over all nodes of the plane) of
   P_zz - (P_xx + P_yy)/2; profile (nz values) may be NULL. */
double ora_surface_tension_z(ora_lattice* L, double* profile);

/* Eq. (mechRadGamma) about centre[3]: shells of unit width (bin b holds
   b <= |x - c| < b + 1, minimum image), profile[b] / phi_profile[b] (nbins
   each, may be NULL) the shell means of P_N - P_T and of phi, *Rs the
   outward phi crossing; returns the sum over shells with b + 1/2 <= rmax of
   ((b + 1/2) / R_s)^2 profile[b], or NaN without a crossing. */
double ora_radial_tension(ora_lattice* L, const double* center, double rmax, int nbins,
                          double* profile, double* phi_profile, double* Rs);
/* The same with the minimum image only along the axes whose bit is set in
   periodic (bit 0 x, bit 1 y, bit 2 z); plain differences along the others. */
double ora_radial_tension_axes(ora_lattice* L, const double* center, int periodic, double rmax,
                               int nbins, double* profile, double* phi_profile, double* Rs);

/* Eq. (young) in degrees from the three tensions (liquid = droplet
   species), clamped to [0, 180]. */
double ora_young_angle(double gamma_sg, double gamma_sl, double gamma_lg);
/* Eq. (huangSigmaLG): Huang's estimate for droplet species A from the wall
   parameters and the A densities of the A-rich (rho_in) and B-rich
   (rho_out) bulk phases; degrees, clamped. */
double ora_huang_angle(const ora_params* p, double rho_in, double rho_out);

/* Host threads of the per-node loops (OpenMP): the count in use, and a
 * setter (n >= 1).  Results do not depend on it: reductions run in a fixed
 * serial order. */
int ora_num_threads(void);
void ora_set_threads(int n);

/* contact angle of the current state; returns 0, or -4 when no droplet */
int ora_contact_angle(const ora_lattice* L, const ora_ca_cfg* cfg, ora_ca* out);
/* same, on a given order-parameter field phi (one value per node); solid
   nodes of the lattice's mask are skipped */
int ora_contact_angle_phi(const ora_lattice* L, const ora_ca_cfg* cfg,
                          const double* phi, ora_ca* out);

/* ---- adjoint (extension: exact transpose of the step) ---- */
/* Seed dtheta_E2 / dC for the current state times dL_dtheta (per radian):
   lam (state layout) is overwritten. */
int ora_ca_seed(const ora_lattice* L, const ora_ca_cfg* cfg, double dL_dtheta, double* lam);
/* One reverse step: state_t is C^t (state layout); lam holds lambda^{t+1} on
   entry and lambda^t on exit.  dparams[5] += dL/d{rho_wall_A, rho_wall_B,
   g_ab, g_wall_A, g_wall_B}. */
void ora_adjoint_step(const ora_lattice* L, const double* state_t, double* lam, double* dparams);

#ifdef __cplusplus
}
#endif
#endif
