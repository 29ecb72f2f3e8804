/*
 * oracle.c -- plain FP64 CPU oracle (test infrastructure only; see oracle.h).
 *
 * Every function follows one passage of the paper and is written as whole-
 * field sub-steps in the order the paper states them, with no blocking or
 * fusion: stream, moments, pseudopotential, force, velocity, collide.
 * Loops over nodes are parallel over z planes (OpenMP); every reduction is a
 * serial loop in a fixed order, so results do not depend on the thread count.
 * Build with -ffp-contract=off so that no multiply-add is fused.
 */
#include "oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* D3Q19 lattice (Sec. 2: "D3Q19 implementation"; zeta_k and c_s are fixed
 * by the lattice).  Velocity order: rest, the six axis vectors in +/- pairs,
 * then the twelve face diagonals in +/- pairs.                              */
static const int CV[ORA_Q][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static const double CS2 = 1.0 / 3.0; /* speed of sound squared of D3Q19 */

static double zeta_from_velocity(int k) {
  int c2 = CV[k][0] * CV[k][0] + CV[k][1] * CV[k][1] + CV[k][2] * CV[k][2];
  if (c2 == 0) return 1.0 / 3.0;
  if (c2 == 1) return 1.0 / 18.0;
  return 1.0 / 36.0;
}

static int opposite_from_velocity(int k) {
  for (int j = 0; j < ORA_Q; ++j)
    if (CV[j][0] == -CV[k][0] && CV[j][1] == -CV[k][1] && CV[j][2] == -CV[k][2]) return j;
  return -1;
}

/* the two tables above, evaluated once, and the coefficients of the
 * equilibrium's expansion in c.u and u^2 (Eq. Equil) in units of c_s */
static double ZETA[ORA_Q];
static int OPP[ORA_Q];
static double E_CU, E_CU2, E_UU, E_CU3, E_UUCU; /* 1/cs2, 1/2cs4, 1/2cs2, 1/6cs6, 1/2cs4 */
static int tables_ready = 0;
static void make_tables(void) {
  if (tables_ready) return;
  for (int k = 0; k < ORA_Q; ++k) {
    ZETA[k] = zeta_from_velocity(k);
    OPP[k] = opposite_from_velocity(k);
  }
  E_CU = 1.0 / CS2;
  E_CU2 = 1.0 / (2.0 * CS2 * CS2);
  E_UU = 1.0 / (2.0 * CS2);
  E_CU3 = 1.0 / (6.0 * CS2 * CS2 * CS2);
  E_UUCU = 1.0 / (2.0 * CS2 * CS2);
  tables_ready = 1;
}
static double zeta_of(int k) { return ZETA[k]; }
static int opposite_of(int k) { return OPP[k]; }

void ora_tables(int32_t* c, double* w, int32_t* opp) {
  make_tables();
  for (int k = 0; k < ORA_Q; ++k) {
    for (int d = 0; d < 3; ++d) c[k * 3 + d] = CV[k][d];
    w[k] = zeta_of(k);
    opp[k] = opposite_of(k);
  }
}

/* Eq. (Equil): third-order equilibrium of one species with velocity u. */
static double equilibrium_k(int k, double rho, const double* u) {
  double cu = CV[k][0] * u[0] + CV[k][1] * u[1] + CV[k][2] * u[2];
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double bracket = 1.0 + E_CU * cu + E_CU2 * (cu * cu) - E_UU * uu + E_CU3 * (cu * cu * cu) -
                   E_UUCU * (uu * cu);
  return zeta_of(k) * rho * bracket;
}

void ora_equilibrium(double rho, const double* u, double* out) {
  make_tables();
  for (int k = 0; k < ORA_Q; ++k) out[k] = equilibrium_k(k, rho, u);
}

/* Sec. 2: pseudopotential psi(rho); the paper's form is 1 - exp(-rho). */
static double psi_of(int form, double rho) { return form == 1 ? 1.0 - exp(-rho) : rho; }
static double dpsi_of(int form, double rho) { return form == 1 ? exp(-rho) : 1.0; }

/* ------------------------------------------------------------------------ */
struct ora_lattice {
  ora_params p;
  int nx, ny, nz;
  size_t N;
  uint8_t* solid;
  double* C;   /* state: post-collision populations, 38 per node */
  double* n;   /* post-stream populations */
  double* rho; /* 2 per node */
  double* j;   /* 6 per node */
  double* psi; /* 2 per node */
  double* F;   /* 6 per node */
  double* u;   /* 6 per node: equilibrium velocity of each species */
  int64_t step;
};

/* periodic wrap of one coordinate */
static int wrap(int x, int n) {
  while (x < 0) x += n;
  while (x >= n) x -= n;
  return x;
}

static size_t node_at(const ora_lattice* L, int x, int y, int z) {
  return ((size_t)wrap(z, L->nz) * L->ny + wrap(y, L->ny)) * L->nx + wrap(x, L->nx);
}

static int params_ok(const ora_params* p) {
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return 0;
  if (!(p->tau[0] > 0.5) || !(p->tau[1] > 0.5)) return 0;
  if (p->psi != 0 && p->psi != 1) return 0;
  return 1;
}

ora_lattice* ora_create(const ora_params* p, const uint8_t* solid) {
  make_tables();
  if (!params_ok(p)) return NULL;
  ora_lattice* L = (ora_lattice*)calloc(1, sizeof(ora_lattice));
  L->p = *p;
  L->nx = p->nx; L->ny = p->ny; L->nz = p->nz;
  L->N = (size_t)p->nx * p->ny * p->nz;
  L->solid = (uint8_t*)calloc(L->N, 1);
  if (solid) for (size_t i = 0; i < L->N; ++i) L->solid[i] = solid[i] ? 1 : 0;
  L->C = (double*)calloc(L->N * 38, sizeof(double));
  L->n = (double*)calloc(L->N * 38, sizeof(double));
  L->rho = (double*)calloc(L->N * 2, sizeof(double));
  L->j = (double*)calloc(L->N * 6, sizeof(double));
  L->psi = (double*)calloc(L->N * 2, sizeof(double));
  L->F = (double*)calloc(L->N * 6, sizeof(double));
  L->u = (double*)calloc(L->N * 6, sizeof(double));
  return L;
}

void ora_destroy(ora_lattice* L) {
  if (!L) return;
  free(L->solid); free(L->C); free(L->n); free(L->rho); free(L->j);
  free(L->psi); free(L->F); free(L->u); free(L);
}

int ora_set_params(ora_lattice* L, const ora_params* p) {
  if (!params_ok(p) || p->nx != L->nx || p->ny != L->ny || p->nz != L->nz) return -1;
  L->p = *p;
  return 0;
}

void ora_init_equilibrium_u(ora_lattice* L, const double* rho_a, const double* rho_b,
                            const double* u) {
  const double zero[3] = {0.0, 0.0, 0.0};
  for (size_t i = 0; i < L->N; ++i) {
    double* c = L->C + i * 38;
    if (L->solid[i]) { memset(c, 0, 38 * sizeof(double)); continue; }
    const double* ui = u ? u + i * 3 : zero;
    for (int k = 0; k < ORA_Q; ++k) {
      c[k] = equilibrium_k(k, rho_a[i], ui);
      c[ORA_Q + k] = equilibrium_k(k, rho_b[i], ui);
    }
  }
  L->step = 0;
}

void ora_init_equilibrium(ora_lattice* L, const double* rho_a, const double* rho_b) {
  ora_init_equilibrium_u(L, rho_a, rho_b, NULL);
}

int64_t ora_step_count(const ora_lattice* L) { return L->step; }

void ora_get_state(const ora_lattice* L, double* dst) {
  memcpy(dst, L->C, L->N * 38 * sizeof(double));
}

void ora_set_state(ora_lattice* L, const double* src) {
  memcpy(L->C, src, L->N * 38 * sizeof(double));
}

/* ------------------------------------------------------------------------ */
/* Sub-step 1, Eq. (LBeqs) streaming with mid-grid bounce-back (Sec. 2 wall
 * model): the population arriving at fluid node x along c_k comes from
 * x - c_k; when that node is solid, the population that left x along the
 * opposite direction is reflected back at the half-way wall.              */
static void stream_field(const ora_lattice* L, const double* in, double* out) {
#pragma omp parallel for schedule(static)
  for (int z = 0; z < L->nz; ++z)
    for (int y = 0; y < L->ny; ++y)
      for (int x = 0; x < L->nx; ++x) {
        size_t i = node_at(L, x, y, z);
        double* o = out + i * 38;
        if (L->solid[i]) { memset(o, 0, 38 * sizeof(double)); continue; }
        for (int k = 0; k < ORA_Q; ++k) {
          size_t src = node_at(L, x - CV[k][0], y - CV[k][1], z - CV[k][2]);
          int kb = opposite_of(k);
          for (int a = 0; a < 2; ++a) {
            if (L->solid[src]) o[a * ORA_Q + k] = in[i * 38 + a * ORA_Q + kb];
            else o[a * ORA_Q + k] = in[src * 38 + a * ORA_Q + k];
          }
        }
      }
}

void ora_stream(const ora_lattice* L, const double* in, double* out) { stream_field(L, in, out); }

/* Sub-step 2, Sec. 2: rho^a = sum_k n_k^a and rho^a u^a = sum_k n_k^a c_k. */
static void moments(ora_lattice* L) {
#pragma omp parallel for schedule(static)
  for (int z = 0; z < L->nz; ++z)
    for (size_t i = (size_t)z * L->nx * L->ny; i < (size_t)(z + 1) * L->nx * L->ny; ++i) {
      for (int a = 0; a < 2; ++a) {
        double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
        if (!L->solid[i]) {
          for (int k = 0; k < ORA_Q; ++k) {
            double f = L->n[i * 38 + a * ORA_Q + k];
            r += f;
            jx += f * CV[k][0];
            jy += f * CV[k][1];
            jz += f * CV[k][2];
          }
        }
        L->rho[i * 2 + a] = r;
        L->j[i * 6 + a * 3 + 0] = jx;
        L->j[i * 6 + a * 3 + 1] = jy;
        L->j[i * 6 + a * 3 + 2] = jz;
      }
    }
}

/* Sub-step 3, Sec. 2: effective mass psi at fluid nodes; at wall nodes the
 * wall acts as an extra species of constant density (its A- and B-content). */
static void pseudopotential(const ora_lattice* L, const double* rho, double* psi) {
  for (size_t i = 0; i < L->N; ++i)
    for (int a = 0; a < 2; ++a)
      psi[i * 2 + a] = L->solid[i] ? psi_of(L->p.psi, L->p.rho_wall[a])
                                   : psi_of(L->p.psi, rho[i * 2 + a]);
}

/* Coupling G^a(y) seen by species a at neighbour y: g_ab between the two
 * fluid species (Eq. SCforce), g_wall^a when y is a wall node (Sec. 2). */
static double coupling(const ora_lattice* L, int a, size_t y) {
  return L->solid[y] ? L->p.g_wall[a] : L->p.g_ab;
}

static double weight_of(const ora_lattice* L, int k) {
  int c2 = CV[k][0] * CV[k][0] + CV[k][1] * CV[k][1] + CV[k][2] * CV[k][2];
  return c2 == 1 ? L->p.w_axis : L->p.w_diag;
}

/* Sub-step 4, Eq. (SCforce): F^a(x) = -psi^a(x) sum over the 18 nearest
 * neighbours x' = x + c_k of G^a(x') psi^b(x') (x' - x), b the other species. */
static void force_field(const ora_lattice* L, const double* psi, double* F) {
#pragma omp parallel for schedule(static)
  for (int z = 0; z < L->nz; ++z)
    for (int y = 0; y < L->ny; ++y)
      for (int x = 0; x < L->nx; ++x) {
        size_t i = node_at(L, x, y, z);
        for (int a = 0; a < 2; ++a) {
          int b = 1 - a;
          double s[3] = {0.0, 0.0, 0.0};
          if (!L->solid[i]) {
            for (int k = 1; k < ORA_Q; ++k) {
              size_t yy = node_at(L, x + CV[k][0], y + CV[k][1], z + CV[k][2]);
              double gp = weight_of(L, k) * coupling(L, a, yy) * psi[yy * 2 + b];
              for (int d = 0; d < 3; ++d) s[d] += gp * CV[k][d];
            }
          }
          for (int d = 0; d < 3; ++d)
            F[i * 6 + a * 3 + d] = L->solid[i] ? 0.0 : -psi[i * 2 + a] * s[d];
        }
      }
}

void ora_force(const ora_lattice* L, const double* rho, double* F) {
  double* psi = (double*)malloc(L->N * 2 * sizeof(double));
  pseudopotential(L, rho, psi);
  force_field(L, psi, F);
  free(psi);
}

/* Sub-step 5, Sec. 2: the common velocity u' of both species (Shan-Chen's
 * relaxation-time weighted mean) plus the shift du^a = tau^a F^a / rho^a. */
static void velocity(ora_lattice* L) {
#pragma omp parallel for schedule(static)
  for (int z = 0; z < L->nz; ++z)
    for (size_t i = (size_t)z * L->nx * L->ny; i < (size_t)(z + 1) * L->nx * L->ny; ++i) {
      if (L->solid[i]) { for (int d = 0; d < 6; ++d) L->u[i * 6 + d] = 0.0; continue; }
      double R = 0.0, J[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < 2; ++a) {
        R += L->rho[i * 2 + a] / L->p.tau[a];
        for (int d = 0; d < 3; ++d) J[d] += L->j[i * 6 + a * 3 + d] / L->p.tau[a];
      }
      for (int a = 0; a < 2; ++a)
        for (int d = 0; d < 3; ++d)
          L->u[i * 6 + a * 3 + d] =
              J[d] / R + L->p.tau[a] * L->F[i * 6 + a * 3 + d] / L->rho[i * 2 + a];
    }
}

/* Sub-step 6, BGK collision (Sec. 2): C' = n - (n - n^eq(rho, u)) / tau. */
static void collide(ora_lattice* L, double* out) {
#pragma omp parallel for schedule(static)
  for (int z = 0; z < L->nz; ++z)
    for (size_t i = (size_t)z * L->nx * L->ny; i < (size_t)(z + 1) * L->nx * L->ny; ++i) {
      double* o = out + i * 38;
      if (L->solid[i]) { memset(o, 0, 38 * sizeof(double)); continue; }
      for (int a = 0; a < 2; ++a)
        for (int k = 0; k < ORA_Q; ++k) {
          double nk = L->n[i * 38 + a * ORA_Q + k];
          double eq = equilibrium_k(k, L->rho[i * 2 + a], L->u + i * 6 + a * 3);
          o[a * ORA_Q + k] = nk - (nk - eq) / L->p.tau[a];
        }
    }
}

/* All sub-steps up to (not including) the collision, from the state C. */
static void forward_fields(ora_lattice* L, const double* C) {
  stream_field(L, C, L->n);
  moments(L);
  pseudopotential(L, L->rho, L->psi);
  force_field(L, L->psi, L->F);
  velocity(L);
}

void ora_step(ora_lattice* L, int64_t nsteps) {
  for (int64_t s = 0; s < nsteps; ++s) {
    forward_fields(L, L->C);
    collide(L, L->C); /* reads only n, rho, u, so writing C in place is safe */
    L->step += 1;
  }
}

/* ------------------------------------------------------------------------ */
/* Pressure tensor of Sec. 4.1 at every node, from the post-stream
 * populations n of the current state (the distribution at time t that the
 * collision acts on).  At a fluid node x:
 *   P_ij(x) = sum_a sum_k (c_ki - u_i)(c_kj - u_j) n_k^a(x)
 *           + 1/2 sum_k W_k c_ki c_kj [psi^A(x) G^A(y) psi^B(y) + psi^B(x) G^B(y) psi^A(y)]
 * with y = x + c_k.  u is the velocity of the fluid, (sum_a j^a + F / 2) /
 * sum_a rho^a with F = sum_a F^a of Eq. (SCforce): the momentum of the
 * populations plus half the momentum the force adds in a step.  With it the
 * normal component of a planar interface at rest is the same on every plane
 * (mechanical equilibrium); with the populations' momentum alone it is not.
 * The paper's second term sums over the ordered species pairs with a
 * prefactor 1/4; both orderings give the same bracket, hence 1/2.  Its pair
 * factor (x - x')^2 is read as the dyad (x - x')_i (x - x')_j of a tensor.
 * Wall neighbours enter as in the force (Sec. 2 wall model): their content
 * through psi and the coupling g_wall^a.
 * At a wall node x (the wall taken as a component of the system, as in the
 * wall slabs of Sec. 4.1) there is no kinetic part and P_ij(x) is the wall's
 * half of every wall-fluid pair, the same pair term seen from the wall:
 *   P_ij(x) = 1/2 sum_{k: y fluid} W_k c_ki c_kj
 *             [g_wall^A psi^A(y) psi(rho_wall^B) + g_wall^B psi^B(y) psi(rho_wall^A)];
 * wall-wall pairs carry no force and add nothing.                          */
void ora_pressure_tensor(ora_lattice* L, double* P) {
  forward_fields(L, L->C);
  static const int PI[6] = {0, 1, 2, 0, 0, 1}, PJ[6] = {0, 1, 2, 1, 2, 2};
#pragma omp parallel for schedule(static)
  for (int z = 0; z < L->nz; ++z)
    for (int y = 0; y < L->ny; ++y)
      for (int x = 0; x < L->nx; ++x) {
        size_t i = node_at(L, x, y, z);
        double* out = P + i * 6;
        for (int c = 0; c < 6; ++c) out[c] = 0.0;
        if (L->solid[i]) {
          for (int c = 0; c < 6; ++c) {
            double inter = 0.0;
            for (int k = 1; k < ORA_Q; ++k) {
              size_t yy = node_at(L, x + CV[k][0], y + CV[k][1], z + CV[k][2]);
              if (L->solid[yy]) continue;
              double br = L->p.g_wall[0] * L->psi[yy * 2] * L->psi[i * 2 + 1] +
                          L->p.g_wall[1] * L->psi[yy * 2 + 1] * L->psi[i * 2];
              inter += weight_of(L, k) * CV[k][PI[c]] * CV[k][PJ[c]] * br;
            }
            out[c] = 0.5 * inter;
          }
          continue;
        }
        double R = L->rho[i * 2] + L->rho[i * 2 + 1];
        double u[3];
        for (int d = 0; d < 3; ++d)
          u[d] = (L->j[i * 6 + d] + L->j[i * 6 + 3 + d] +
                  0.5 * (L->F[i * 6 + d] + L->F[i * 6 + 3 + d])) / R;
        for (int c = 0; c < 6; ++c) {
          double kin = 0.0, inter = 0.0;
          for (int k = 0; k < ORA_Q; ++k) {
            double nk = L->n[i * 38 + k] + L->n[i * 38 + ORA_Q + k];
            kin += (CV[k][PI[c]] - u[PI[c]]) * (CV[k][PJ[c]] - u[PJ[c]]) * nk;
          }
          for (int k = 1; k < ORA_Q; ++k) {
            size_t yy = node_at(L, x + CV[k][0], y + CV[k][1], z + CV[k][2]);
            double br = L->psi[i * 2] * coupling(L, 0, yy) * L->psi[yy * 2 + 1] +
                        L->psi[i * 2 + 1] * coupling(L, 1, yy) * L->psi[yy * 2];
            inter += weight_of(L, k) * CV[k][PI[c]] * CV[k][PJ[c]] * br;
          }
          out[c] = kin + 0.5 * inter;
        }
      }
}

/* Eq. (gammaMechDef) on the lattice for interfaces normal to z: the sum over
 * the planes z of the plane mean (over all its nodes, fluid and wall) of
 * P_N - P_T = P_zz - (P_xx + P_yy) / 2.  A periodic box with two interfaces
 * holds twice the surface tension.  profile (nz values, or NULL): the plane
 * means.                                                                   */
double ora_surface_tension_z(ora_lattice* L, double* profile) {
  double* P = (double*)malloc(L->N * 6 * sizeof(double));
  ora_pressure_tensor(L, P);
  double total = 0.0;
  size_t A = (size_t)L->nx * L->ny;
  for (int z = 0; z < L->nz; ++z) {
    double s = 0.0;
    for (size_t i = (size_t)z * A; i < (size_t)(z + 1) * A; ++i)
      s += P[i * 6 + 2] - 0.5 * (P[i * 6 + 0] + P[i * 6 + 1]);
    double m = s / (double)A;
    if (profile) profile[z] = m;
    total += m;
  }
  free(P);
  return total;
}

/* ------------------------------------------------------------------------ */
void ora_density(const ora_lattice* L, double* rho) {
  for (size_t i = 0; i < L->N; ++i)
    for (int a = 0; a < 2; ++a) {
      double r = 0.0;
      if (!L->solid[i])
        for (int k = 0; k < ORA_Q; ++k) r += L->C[i * 38 + a * ORA_Q + k];
      rho[i * 2 + a] = r;
    }
}

void ora_observables(const ora_lattice* L, double* out) {
  double m[2] = {0.0, 0.0}, P[3] = {0.0, 0.0, 0.0};
  int finite = 1;
  for (size_t i = 0; i < L->N; ++i) {
    if (L->solid[i]) continue;
    for (int a = 0; a < 2; ++a)
      for (int k = 0; k < ORA_Q; ++k) {
        double f = L->C[i * 38 + a * ORA_Q + k];
        if (!isfinite(f)) finite = 0;
        m[a] += f;
        for (int d = 0; d < 3; ++d) P[d] += f * CV[k][d];
      }
  }
  out[0] = m[0]; out[1] = m[1];
  out[2] = P[0]; out[3] = P[1]; out[4] = P[2];
  out[5] = finite ? 1.0 : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Contact angle, Sec. 3 (Eq. geoCA) and the smoothed-indicator variant.     */
typedef struct {
  const ora_lattice* L;
  const double* phi;
} phi_view;

static int is_solid(const phi_view* v, int x, int y, int z) {
  if (z < 0 || z >= v->L->nz) return 1;
  return v->L->solid[node_at(v->L, x, y, z)];
}
static double phi_at(const phi_view* v, int x, int y, int z) {
  return v->phi[node_at(v->L, x, y, z)];
}

/* First crossing of phi from > 0 to <= 0 going up the column from k0;
 * linear interpolation between the two nodes.  NaN when none is found. */
static double apex_crossing(const phi_view* v, int ic, int jc, int k0) {
  for (int k = k0; k + 1 < v->L->nz; ++k) {
    if (is_solid(v, ic, jc, k + 1)) break;
    double p0 = phi_at(v, ic, jc, k), p1 = phi_at(v, ic, jc, k + 1);
    if (p0 > 0.0 && p1 <= 0.0) return k + p0 / (p0 - p1);
  }
  return NAN;
}

/* Half-chord from the column along (sx, sy) in layer k: distance to the
 * first phi crossing; rays stop at half the box length. */
static double half_chord(const phi_view* v, int ic, int jc, int k, int sx, int sy, int* flags) {
  int len = sx != 0 ? v->L->nx : v->L->ny;
  for (int m = 0; m < len / 2; ++m) {
    double p0 = phi_at(v, ic + m * sx, jc + m * sy, k);
    double p1 = phi_at(v, ic + (m + 1) * sx, jc + (m + 1) * sy, k);
    if (p0 > 0.0 && p1 <= 0.0) return m + p0 / (p0 - p1);
  }
  *flags |= ORA_CA_RAY_LIMIT;
  return len / 2;
}

static double mean_half_chord(const phi_view* v, int ic, int jc, int k, int* flags) {
  return 0.25 * (half_chord(v, ic, jc, k, 1, 0, flags) + half_chord(v, ic, jc, k, -1, 0, flags) +
                 half_chord(v, ic, jc, k, 0, 1, flags) + half_chord(v, ic, jc, k, 0, -1, flags));
}

static const double RAD2DEG = 57.295779513082320876798154814105;

/* Cap through a circle of half-width aref at the reference plane and an apex
 * H above that plane: sphere radius R = (aref^2 + H^2) / 2H (Sec. 3, the
 * relation r = (4h^2 + b^2)/8h taken relative to the reference plane).  The
 * base half-width at the wall then follows from a^2 = 2Rh - h^2 and the
 * contact angle is theta = 2 atan(h / a), which is Eq. (geoCA) with the
 * branch chosen so that flat caps give angles below 90 degrees. */
static double cap_angle(double aref2, double H, double h, double* R, double* a, int* flat) {
  *R = (aref2 + H * H) / (2.0 * H);
  double a2 = 2.0 * (*R) * h - h * h;
  if (!(a2 > 0.0)) { *flat = 1; *a = 0.0; return 180.0; }
  *flat = 0;
  *a = sqrt(a2);
  return 2.0 * atan2(h, *a) * RAD2DEG;
}

static double smoothstep(double t) {
  if (t <= 0.0) return 0.0;
  if (t >= 1.0) return 1.0;
  return t * t * (3.0 - 2.0 * t);
}
static double dsmoothstep(double t) {
  if (t <= 0.0 || t >= 1.0) return 0.0;
  return 6.0 * t * (1.0 - t);
}

/* Smoothed droplet indicator of the order parameter (0 at solid nodes). */
static double indicator(const phi_view* v, double eps, int x, int y, int z) {
  if (is_solid(v, x, y, z)) return 0.0;
  return smoothstep((phi_at(v, x, y, z) + eps) / (2.0 * eps));
}
static double dindicator(const phi_view* v, double eps, int x, int y, int z) {
  if (is_solid(v, x, y, z)) return 0.0;
  return dsmoothstep((phi_at(v, x, y, z) + eps) / (2.0 * eps)) / (2.0 * eps);
}

/* Top of the droplet's run of the column: the first node above kref where
 * the indicator vanishes (or a solid node).  Anything above it (a film on
 * the ceiling, another droplet) is not part of this droplet. */
static int e2_column_end(const phi_view* v, const ora_ca_cfg* cfg) {
  int kref = cfg->z_solid_top + cfg->offset;
  int k = kref + 1;
  while (k < v->L->nz && indicator(v, cfg->eps, cfg->ic, cfg->jc, k) > 0.0) ++k;
  return k;
}

/* Radius of the disk around the column over which E2 sums the reference
 * layer: the largest E1 half-chord in that layer plus 4 lattice units (the
 * indicator's transition band), so that other A-rich regions of the layer
 * (a film on the wall, a second droplet) are not counted.  Without a droplet
 * at the reference layer the whole layer is used (flag E2_WHOLE_LAYER). */
static double e2_window(const phi_view* v, const ora_ca_cfg* cfg, int* flags) {
  int kref = cfg->z_solid_top + cfg->offset;
  if (!(phi_at(v, cfg->ic, cfg->jc, kref) > 0.0)) {
    *flags |= ORA_CA_E2_WHOLE_LAYER;
    return INFINITY;
  }
  int f = 0;
  double r = half_chord(v, cfg->ic, cfg->jc, kref, 1, 0, &f);
  double t = half_chord(v, cfg->ic, cfg->jc, kref, -1, 0, &f);
  if (t > r) r = t;
  t = half_chord(v, cfg->ic, cfg->jc, kref, 0, 1, &f);
  if (t > r) r = t;
  t = half_chord(v, cfg->ic, cfg->jc, kref, 0, -1, &f);
  if (t > r) r = t;
  return r + 4.0;
}

/* periodic (minimum image) distance along one axis */
static int image_dist(int a, int b, int n) {
  int d = a > b ? a - b : b - a;
  return d < n - d ? d : n - d;
}

static int in_window(const phi_view* v, const ora_ca_cfg* cfg, double rcut, int x, int y) {
  double dx = image_dist(x, cfg->ic, v->L->nx), dy = image_dist(y, cfg->jc, v->L->ny);
  return dx * dx + dy * dy <= rcut * rcut;
}

/* E2 column and layer sums: H = 1/2 chi(kref) + sum_{kref < k < kend} chi
 * and A = sum over the reference layer window of chi / pi (area / pi =
 * aref^2). */
static void e2_sums(const phi_view* v, const ora_ca_cfg* cfg, double rcut, double* H, double* A) {
  int kref = cfg->z_solid_top + cfg->offset;
  int kend = e2_column_end(v, cfg);
  double h = 0.5 * indicator(v, cfg->eps, cfg->ic, cfg->jc, kref);
  for (int k = kref + 1; k < kend; ++k) h += indicator(v, cfg->eps, cfg->ic, cfg->jc, k);
  double s = 0.0;
  for (int y = 0; y < v->L->ny; ++y)
    for (int x = 0; x < v->L->nx; ++x)
      if (in_window(v, cfg, rcut, x, y)) s += indicator(v, cfg->eps, x, y, kref);
  *H = h;
  *A = s / M_PI;
}

int ora_contact_angle_phi(const ora_lattice* L, const ora_ca_cfg* cfg, const double* phi,
                          ora_ca* out) {
  phi_view v = {L, phi};
  memset(out, 0, sizeof(*out));
  int ic = cfg->ic, jc = cfg->jc, zs = cfg->z_solid_top;
  int kref = zs + cfg->offset;
  double zw = zs + 0.5; /* mid-grid wall: half a spacing above the solid layer */
  double d = kref - zw;
  int flags = 0;

  /* centroid of phi > 0 in the reference layer */
  double sx = 0.0, sy = 0.0, cnt = 0.0;
  for (int y = 0; y < L->ny; ++y)
    for (int x = 0; x < L->nx; ++x)
      if (!is_solid(&v, x, y, kref) && phi_at(&v, x, y, kref) > 0.0) { sx += x; sy += y; cnt += 1.0; }
  out->cx = cnt > 0.0 ? sx / cnt : NAN;
  out->cy = cnt > 0.0 ? sy / cnt : NAN;

  if (!(phi_at(&v, ic, jc, zs + 1) > 0.0)) {
    flags |= ORA_CA_NO_DROP;
    out->theta_e1 = out->theta_e2 = NAN;
    out->flags = flags;
    return -4;
  }

  /* E1: zero crossings of phi (Sec. 3) */
  int flat = 0;
  if (phi_at(&v, ic, jc, kref) > 0.0) {
    double ztop = apex_crossing(&v, ic, jc, kref);
    if (isnan(ztop)) {
      flags |= ORA_CA_NO_APEX;
      out->theta_e1 = NAN;
    } else {
      double h = ztop - zw, H = ztop - kref;
      double aref = mean_half_chord(&v, ic, jc, kref, &flags);
      double R, a;
      out->theta_e1 = cap_angle(aref * aref, H, h, &R, &a, &flat);
      if (flat) flags |= ORA_CA_E1_FLAT;
      out->h_e1 = h; out->H_e1 = H; out->aref_e1 = aref; out->R_e1 = R; out->a_e1 = a;
    }
  } else {
    /* droplet flatter than the reference plane: measure the base directly in
       the first fluid layer and the height from the apex */
    flags |= ORA_CA_NO_REF;
    double ztop = apex_crossing(&v, ic, jc, zs + 1);
    if (isnan(ztop)) {
      flags |= ORA_CA_NO_APEX;
      out->theta_e1 = NAN;
    } else {
      double h = ztop - zw;
      double a = mean_half_chord(&v, ic, jc, zs + 1, &flags);
      out->theta_e1 = 2.0 * atan2(h, a) * RAD2DEG;
      out->h_e1 = h; out->a_e1 = a; out->H_e1 = ztop - kref; out->aref_e1 = NAN;
      out->R_e1 = (a * a + h * h) / (2.0 * h);
    }
  }

  /* E2: smoothed indicator sums */
  double H, A;
  double rcut = e2_window(&v, cfg, &flags);
  e2_sums(&v, cfg, rcut, &H, &A);
  out->H_e2 = H;
  out->aref_e2 = sqrt(A);
  if (!(H > 0.0)) {
    flags |= ORA_CA_E2_EMPTY;
    out->theta_e2 = NAN;
  } else {
    double h = H + d, R, a;
    out->theta_e2 = cap_angle(A, H, h, &R, &a, &flat);
    if (flat) flags |= ORA_CA_E2_FLAT;
    out->h_e2 = h; out->R_e2 = R; out->a_e2 = a;
  }
  out->flags = flags;
  return 0;
}

int ora_contact_angle(const ora_lattice* L, const ora_ca_cfg* cfg, ora_ca* out) {
  double* rho = (double*)malloc(L->N * 2 * sizeof(double));
  double* phi = (double*)malloc(L->N * sizeof(double));
  ora_density(L, rho);
  for (size_t i = 0; i < L->N; ++i) phi[i] = rho[i * 2 + 0] - rho[i * 2 + 1]; /* Sec. 2 */
  int rc = ora_contact_angle_phi(L, cfg, phi, out);
  free(rho);
  free(phi);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Adjoint.  Seed: derivative of theta_E2 (radians) with respect to every
 * population of the state, times dL/dtheta.  theta depends on the state only
 * through phi = rho_A - rho_B = sum_k C_k^A - sum_k C_k^B. */
int ora_ca_seed(const ora_lattice* L, const ora_ca_cfg* cfg, double dL_dtheta, double* lam) {
  double* rho = (double*)malloc(L->N * 2 * sizeof(double));
  double* phi = (double*)malloc(L->N * sizeof(double));
  ora_density(L, rho);
  for (size_t i = 0; i < L->N; ++i) phi[i] = rho[i * 2 + 0] - rho[i * 2 + 1];
  phi_view v = {L, phi};
  memset(lam, 0, L->N * 38 * sizeof(double));
  int kref = cfg->z_solid_top + cfg->offset;
  double d = kref - (cfg->z_solid_top + 0.5);
  double H, A;
  int wflags = 0;
  double rcut = e2_window(&v, cfg, &wflags);
  e2_sums(&v, cfg, rcut, &H, &A);
  int rc = 0;
  if (H > 0.0) {
    double h = H + d;
    double a2 = (A + H * H) * h / H - h * h;
    if (a2 > 0.0) {
      double a = sqrt(a2);
      /* a^2 = (A + H^2) h / H - h^2 with h = H + d */
      double da2_dA = h / H;
      double da2_dH = ((2.0 * H * h + (A + H * H)) * H - (A + H * H) * h) / (H * H) - 2.0 * h;
      double den = a2 + h * h;
      double dth_dH = 2.0 * (a - h * da2_dH / (2.0 * a)) / den;
      double dth_dA = 2.0 * (-h * da2_dA / (2.0 * a)) / den;
      double* g = (double*)calloc(L->N, sizeof(double)); /* dtheta/dphi */
      for (int y = 0; y < L->ny; ++y)
        for (int x = 0; x < L->nx; ++x)
          if (in_window(&v, cfg, rcut, x, y))
            g[node_at(L, x, y, kref)] += dth_dA * dindicator(&v, cfg->eps, x, y, kref) / M_PI;
      g[node_at(L, cfg->ic, cfg->jc, kref)] +=
          0.5 * dth_dH * dindicator(&v, cfg->eps, cfg->ic, cfg->jc, kref);
      int kend = e2_column_end(&v, cfg);
      for (int k = kref + 1; k < kend; ++k)
        g[node_at(L, cfg->ic, cfg->jc, k)] += dth_dH * dindicator(&v, cfg->eps, cfg->ic, cfg->jc, k);
      for (size_t i = 0; i < L->N; ++i) {
        if (L->solid[i] || g[i] == 0.0) continue;
        for (int k = 0; k < ORA_Q; ++k) {
          lam[i * 38 + k] = dL_dtheta * g[i];
          lam[i * 38 + ORA_Q + k] = -dL_dtheta * g[i];
        }
      }
      free(g);
    }
  } else {
    rc = -4;
  }
  free(rho);
  free(phi);
  return rc;
}

/* One reverse step: the transposes of sub-steps 6, 5, 4, 3, 2, 1 in that
 * order, applied to lambda^{t+1} = dL/dC^{t+1}. */
void ora_adjoint_step(const ora_lattice* Lc, const double* state_t, double* lam, double* dparams) {
  ora_lattice* L = (ora_lattice*)Lc; /* work fields are scratch */
  const size_t N = L->N;
  forward_fields(L, state_t);

  double* dn = (double*)calloc(N * 38, sizeof(double));
  double* drho = (double*)calloc(N * 2, sizeof(double));
  double* dj = (double*)calloc(N * 6, sizeof(double));
  double* dpsi = (double*)calloc(N * 2, sizeof(double));
  double* dF = (double*)calloc(N * 6, sizeof(double));
  double* du = (double*)calloc(N * 6, sizeof(double));

  /* 6^T collision: C' = n (1 - 1/tau) + n^eq(rho, u) / tau */
  for (size_t i = 0; i < N; ++i) {
    if (L->solid[i]) continue;
    for (int a = 0; a < 2; ++a) {
      double tau = L->p.tau[a], rho = L->rho[i * 2 + a];
      const double* u = L->u + i * 6 + a * 3;
      double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
      for (int k = 0; k < ORA_Q; ++k) {
        double lk = lam[i * 38 + a * ORA_Q + k];
        dn[i * 38 + a * ORA_Q + k] += lk * (1.0 - 1.0 / tau);
        double gk = lk / tau;
        double s = CV[k][0] * u[0] + CV[k][1] * u[1] + CV[k][2] * u[2];
        /* bracket P(s, uu) of Eq. (Equil) and its partial derivatives */
        double P = 1.0 + E_CU * s + E_CU2 * (s * s) - E_UU * uu + E_CU3 * (s * s * s) -
                   E_UUCU * (uu * s);
        double dP_ds = E_CU + 2.0 * E_CU2 * s + 3.0 * E_CU3 * (s * s) - E_UUCU * uu;
        double dP_duu = -E_UU - E_UUCU * s;
        drho[i * 2 + a] += gk * zeta_of(k) * P;
        for (int d = 0; d < 3; ++d)
          du[i * 6 + a * 3 + d] += gk * zeta_of(k) * rho * (dP_ds * CV[k][d] + dP_duu * 2.0 * u[d]);
      }
    }
  }

  /* 5^T velocity: u^a = J/R + tau^a F^a / rho^a */
  for (size_t i = 0; i < N; ++i) {
    if (L->solid[i]) continue;
    double R = 0.0, J[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < 2; ++a) {
      R += L->rho[i * 2 + a] / L->p.tau[a];
      for (int d = 0; d < 3; ++d) J[d] += L->j[i * 6 + a * 3 + d] / L->p.tau[a];
    }
    double dup[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < 2; ++a) {
      double tau = L->p.tau[a], rho = L->rho[i * 2 + a];
      double Fdu = 0.0;
      for (int d = 0; d < 3; ++d) {
        double dua = du[i * 6 + a * 3 + d];
        dF[i * 6 + a * 3 + d] = tau / rho * dua;
        Fdu += L->F[i * 6 + a * 3 + d] * dua;
        dup[d] += dua;
      }
      drho[i * 2 + a] += -tau * Fdu / (rho * rho);
    }
    double dup_up = 0.0;
    for (int d = 0; d < 3; ++d) dup_up += dup[d] * (J[d] / R);
    for (int a = 0; a < 2; ++a) {
      for (int d = 0; d < 3; ++d) dj[i * 6 + a * 3 + d] += dup[d] / (L->p.tau[a] * R);
      drho[i * 2 + a] += -dup_up / (L->p.tau[a] * R);
    }
  }

  /* 4^T force: F^a(x) = -psi^a(x) sum_k W_k G^a(x+c_k) psi^b(x+c_k) c_k */
  for (int z = 0; z < L->nz; ++z)
    for (int y = 0; y < L->ny; ++y)
      for (int x = 0; x < L->nx; ++x) {
        size_t i = node_at(L, x, y, z);
        if (L->solid[i]) continue;
        for (int a = 0; a < 2; ++a) {
          int b = 1 - a;
          const double* dFa = dF + i * 6 + a * 3;
          double s[3] = {0.0, 0.0, 0.0};
          for (int k = 1; k < ORA_Q; ++k) {
            size_t yy = node_at(L, x + CV[k][0], y + CV[k][1], z + CV[k][2]);
            double W = weight_of(L, k), G = coupling(L, a, yy);
            for (int d = 0; d < 3; ++d) s[d] += W * G * L->psi[yy * 2 + b] * CV[k][d];
            double dFc = dFa[0] * CV[k][0] + dFa[1] * CV[k][1] + dFa[2] * CV[k][2];
            double t = -L->psi[i * 2 + a] * W * dFc; /* dL / d(G psi^b)(yy) */
            if (L->solid[yy]) {
              dparams[3 + a] += L->psi[yy * 2 + b] * t;
              dparams[b] += G * t * dpsi_of(L->p.psi, L->p.rho_wall[b]);
            } else {
              dparams[2] += L->psi[yy * 2 + b] * t;
              dpsi[yy * 2 + b] += G * t;
            }
          }
          dpsi[i * 2 + a] += -(dFa[0] * s[0] + dFa[1] * s[1] + dFa[2] * s[2]);
        }
      }

  /* 3^T pseudopotential, 2^T moments, 1^T streaming */
  for (size_t i = 0; i < N; ++i) {
    if (L->solid[i]) continue;
    for (int a = 0; a < 2; ++a) {
      drho[i * 2 + a] += dpsi_of(L->p.psi, L->rho[i * 2 + a]) * dpsi[i * 2 + a];
      for (int k = 0; k < ORA_Q; ++k)
        dn[i * 38 + a * ORA_Q + k] += drho[i * 2 + a] + dj[i * 6 + a * 3 + 0] * CV[k][0] +
                                      dj[i * 6 + a * 3 + 1] * CV[k][1] +
                                      dj[i * 6 + a * 3 + 2] * CV[k][2];
    }
  }
  memset(lam, 0, N * 38 * sizeof(double));
  for (int z = 0; z < L->nz; ++z)
    for (int y = 0; y < L->ny; ++y)
      for (int x = 0; x < L->nx; ++x) {
        size_t i = node_at(L, x, y, z);
        if (L->solid[i]) continue;
        for (int k = 0; k < ORA_Q; ++k) {
          size_t src = node_at(L, x - CV[k][0], y - CV[k][1], z - CV[k][2]);
          int kb = opposite_of(k);
          for (int a = 0; a < 2; ++a) {
            double g = dn[i * 38 + a * ORA_Q + k];
            if (L->solid[src]) lam[i * 38 + a * ORA_Q + kb] += g;
            else lam[src * 38 + a * ORA_Q + k] += g;
          }
        }
      }
  free(dn); free(drho); free(dj); free(dpsi); free(dF); free(du);
}

/* ------------------------------------------------------------------------ */
/* Eq. (mechRadGamma): gamma = int_0^rmax (r / R_s)^2 (P_N - P_T) dr about a
 * centre c (Sec. 4.1).  The integral is a sum over shells of unit width:
 * shell b holds the fluid nodes with b <= |x - c| < b + 1 (minimum-image
 * distances on the periodic axes), at radius r_b = b + 1/2.  P_N = d.P.d / |d|^2
 * and P_T = (tr P - P_N) / 2 with d = x - c; the node at the centre itself
 * adds 0.  profile[b] is the shell mean of P_N - P_T, phi_profile[b] that of
 * phi = rho_A - rho_B.  R_s is the first outward crossing of the shell means
 * of phi from > 0 to <= 0, linearly interpolated between shell radii; the
 * sum runs over the shells with r_b <= rmax.  Returns gamma, or NaN (and
 * R_s = NaN) when phi has no such crossing.                                */
static double min_image(double d, int n) {
  if (d >= 0.5 * n) d -= n;
  if (d < -0.5 * n) d += n;
  return d;
}

double ora_radial_tension(ora_lattice* L, const double* center, double rmax, int nbins,
                          double* profile, double* phi_profile, double* Rs) {
  return ora_radial_tension_axes(L, center, 7, rmax, nbins, profile, phi_profile, Rs);
}

/* The same with the minimum image only along the axes whose bit is set in
 * periodic (bit 0 x, bit 1 y, bit 2 z).  A droplet in the droplet system of
 * Sec. 4.1 rests on a wall: along the wall normal the box is bounded, and
 * the distance from the droplet's centre is the plain difference.          */
double ora_radial_tension_axes(ora_lattice* L, const double* center, int periodic, double rmax,
                               int nbins, double* profile, double* phi_profile, double* Rs) {
  double* P = (double*)malloc(L->N * 6 * sizeof(double));
  double* rho = (double*)malloc(L->N * 2 * sizeof(double));
  double* sv = (double*)calloc((size_t)nbins, sizeof(double));
  double* sp = (double*)calloc((size_t)nbins, sizeof(double));
  double* cnt = (double*)calloc((size_t)nbins, sizeof(double));
  ora_pressure_tensor(L, P);
  ora_density(L, rho);
  for (int z = 0; z < L->nz; ++z)
    for (int y = 0; y < L->ny; ++y)
      for (int x = 0; x < L->nx; ++x) {
        size_t i = node_at(L, x, y, z);
        if (L->solid[i]) continue;
        double d[3] = {x - center[0], y - center[1], z - center[2]};
        const int n[3] = {L->nx, L->ny, L->nz};
        for (int a = 0; a < 3; ++a)
          if ((periodic >> a) & 1) d[a] = min_image(d[a], n[a]);
        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        int b = (int)floor(sqrt(r2));
        while ((double)(b + 1) * (b + 1) <= r2) ++b;
        while (b > 0 && (double)b * b > r2) --b;
        if (b >= nbins) continue;
        const double* p = P + i * 6;
        double v = 0.0;
        if (r2 > 0.0) {
          double pn = (d[0] * d[0] * p[0] + d[1] * d[1] * p[1] + d[2] * d[2] * p[2] +
                       2.0 * (d[0] * d[1] * p[3] + d[0] * d[2] * p[4] + d[1] * d[2] * p[5])) / r2;
          double pt = 0.5 * (p[0] + p[1] + p[2] - pn);
          v = pn - pt;
        }
        sv[b] += v;
        sp[b] += rho[i * 2] - rho[i * 2 + 1];
        cnt[b] += 1.0;
      }
  for (int b = 0; b < nbins; ++b) {
    sv[b] = cnt[b] > 0 ? sv[b] / cnt[b] : 0.0;
    sp[b] = cnt[b] > 0 ? sp[b] / cnt[b] : 0.0;
    if (profile) profile[b] = sv[b];
    if (phi_profile) phi_profile[b] = sp[b];
  }
  double R = NAN;
  for (int b = 0; b + 1 < nbins; ++b)
    if (sp[b] > 0.0 && sp[b + 1] <= 0.0) {
      R = (b + 0.5) + sp[b] / (sp[b] - sp[b + 1]);
      break;
    }
  double g = NAN;
  if (!isnan(R)) {
    g = 0.0;
    for (int b = 0; b < nbins && b + 0.5 <= rmax; ++b) {
      double rb = b + 0.5;
      g += (rb / R) * (rb / R) * sv[b];
    }
  }
  *Rs = R;
  free(P);
  free(rho);
  free(sv);
  free(sp);
  free(cnt);
  return g;
}

/* ------------------------------------------------------------------------ */
/* Eq. (young): cos(theta) = (gamma_SG - gamma_SL) / gamma_LG, the droplet
 * species being the liquid.  Returns theta in degrees, clamped to [0, 180]
 * when |cos| > 1 (complete wetting or drying).                             */
double ora_young_angle(double gamma_sg, double gamma_sl, double gamma_lg) {
  double c = (gamma_sg - gamma_sl) / gamma_lg;
  if (c > 1.0) c = 1.0;
  if (c < -1.0) c = -1.0;
  return acos(c) * RAD2DEG;
}

/* Eq. (huangSigmaLG), Huang's a-priori estimate for droplet species A:
 * cos(theta) = (G_ads,B - G_ads,A) / (g_ab (rho_in - rho_out) / 2), with
 * G_ads,a = g_wall^a psi(rho_wall^b) the adhesion (a repulsion) that species
 * a feels from the wall, and rho_in, rho_out the A densities of the A-rich
 * and B-rich bulk phases.  Clamped as above.                               */
double ora_huang_angle(const ora_params* p, double rho_in, double rho_out) {
  double gA = p->g_wall[0] * psi_of(p->psi, p->rho_wall[1]);
  double gB = p->g_wall[1] * psi_of(p->psi, p->rho_wall[0]);
  return ora_young_angle(gB, gA, p->g_ab * (rho_in - rho_out) / 2.0);
}

int ora_num_threads(void) { return omp_get_max_threads(); }

void ora_set_threads(int n) {
  if (n >= 1) omp_set_num_threads(n);
}
