/*
 * scdrop.h -- C ABI of libscdrop, the MI355X (gfx950) engine for the
 * two-component Shan-Chen lattice Boltzmann model on a D3Q19 lattice with
 * interacting walls, and for the contact-angle observable measured on it.
 *
 * Method (Schmieschek & Harting, "Contact angle determination in
 * multicomponent lattice Boltzmann simulations"):
 *   Sec. 2, Eq. (LBeqs)    per-species streaming + BGK collision
 *   Sec. 2, Eq. (Equil)    third-order equilibrium on D3Q19 (c_s^2 = 1/3)
 *   Sec. 2, Eq. (SCforce)  Shan-Chen force over the 18 nearest neighbours,
 *                          psi = rho (default) or psi = 1 - exp(-rho)
 *   Sec. 2, velocity shift du^a = tau^a F^a / rho^a in the equilibrium
 *   Sec. 2, walls          mid-grid bounce-back; wall nodes act as a species
 *                          of constant density with its own coupling
 *   Sec. 2, order param.   phi = rho_A - rho_B, interface at phi = 0
 *   Sec. 3, Eq. (geoCA)    contact angle from the height and base of the cap,
 *                          measured against a reference layer above the wall
 * The adjoint step, the checkpointed gradient driver and the batched launch
 * are extensions beyond the paper.
 *
 * Conventions
 *   - Node index i = (z * ny + y) * nx + x, x fastest; N = nx * ny * nz.
 *     All three axes are periodic; walls come only from the solid mask.
 *   - Populations C^a_k(x) for species a in {0 = A, 1 = B} and velocity k in
 *     the order: rest; +x, -x, +y, -y, +z, -z;
 *     (+1,+1,0), (-1,-1,0), (+1,-1,0), (-1,+1,0), (+1,0,+1), (-1,0,-1),
 *     (+1,0,-1), (-1,0,+1), (0,+1,+1), (0,-1,-1), (0,+1,-1), (0,-1,+1).
 *     Element type double (SCD_F64) or float (SCD_F32).  The stored state is
 *     post-collision; entries at solid nodes are never read.
 *   - "pop" layout (every population buffer the library reads or writes:
 *     the state, checkpoints, the adjoint's lambda): blocked.  With
 *     P = nx * ny, plane index c = y * nx + x, pb = ceil(P / 32) blocks per
 *     plane and sp = 19 * 32 * pb * nz elements per species, element
 *     (a, k, x, y, z) sits at
 *         a * sp + ((z * pb + c / 32) * 19 + k) * 32 + c % 32.
 *     A buffer holds 2 * sp elements (scd_sizes); the slots past P in the
 *     last block of each plane are padding, never read.
 *   - "plain" layout: structure of arrays, element (a * 19 + k) * N + i,
 *     2 * 19 * N elements.  scd_pop_pack / scd_pop_unpack convert.
 *   - Density arrays are double, 2 * N elements, rho[a * N + i].
 *   - "d_" pointers are device pointers on the current HIP device; "h_"
 *     pointers are host pointers.  The caller allocates every device buffer
 *     and keeps it alive while a handle uses it; the library allocates only
 *     its small host-side handle and never frees caller memory.
 *   - All work is enqueued on the handle's stream in order.  Calls that
 *     return results to the host (observables, contact angle, gradients)
 *     synchronise that stream.
 *   - A handle is not thread-safe; distinct handles may be used from
 *     different threads.
 *   - Every call returns a status; on failure scd_last_error() gives a
 *     message (thread-local, valid until the next call on that thread).
 */
#ifndef SCDROP_H
#define SCDROP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t scd_status;
#define SCD_OK 0
#define SCD_EINVAL (-1)        /* bad argument or parameter */
#define SCD_EDEVICE (-2)       /* HIP runtime error */
#define SCD_ENONFINITE (-3)    /* NaN or Inf in the state */
#define SCD_ENOINTERFACE (-4)  /* no droplet on the measurement column */
#define SCD_EUNSUPPORTED (-5)  /* valid request this build cannot serve */
#define SCD_EDRIFT (-6)        /* mass drifted beyond the watchdog tolerance */

#define SCD_F64 0
#define SCD_F32 1

#define SCD_PSI_RHO 0          /* psi(rho) = rho */
#define SCD_PSI_EXP 1          /* psi(rho) = 1 - exp(-rho), the paper's form */

#define SCD_WITH_ADJOINT 1     /* scd_params.flags: reserve adjoint scratch */

typedef struct {
  int32_t nx, ny, nz;          /* each >= 1; sp * sizeof(real) < 4 GiB
                                  (sp: elements per species, see above) */
  int32_t dtype;               /* SCD_F64 or SCD_F32 */
  int32_t psi;                 /* SCD_PSI_RHO or SCD_PSI_EXP */
  int32_t flags;               /* SCD_WITH_ADJOINT or 0 */
  double tau[2];               /* relaxation times of A and B, > 1/2;
                                  kinematic viscosity (2 tau - 1)/6 (Sec. 4) */
  double g_ab;                 /* fluid-fluid coupling, >= 0 (repulsive) */
  double g_wall[2];            /* coupling felt by A and by B at wall nodes */
  double rho_wall[2];          /* wall content of A and of B, >= 0: species a
                                  feels the other species' wall content */
  double w_axis, w_diag;       /* per-direction weights of the force sum;
                                  1, 1 is the paper's unweighted sum */
} scd_params;

typedef struct {
  double mass[2];              /* sum over fluid nodes of rho^A, rho^B (FP64) */
  double momentum[3];          /* sum over fluid nodes and species of C_k c_k */
  int32_t finite;              /* 1 if every population is finite */
  int32_t pad;
  int64_t step;                /* steps taken since scd_init_equilibrium */
} scd_obs;

typedef struct {
  int32_t ic, jc;              /* column through the droplet axis */
  int32_t z_solid_top;         /* top solid layer under the droplet; the wall
                                  surface is half a spacing above it */
  int32_t offset;              /* reference layer = z_solid_top + offset (5) */
  double eps;                  /* half width of the smoothed indicator (0.2) */
} scd_ca_cfg;

typedef struct {
  /* E1: zero crossings of phi (Sec. 3) */
  double theta_e1, h_e1, a_e1, R_e1, aref_e1, H_e1;
  /* E2: smoothed indicator chi = S((phi + eps) / 2 eps), differentiable */
  double theta_e2, h_e2, a_e2, R_e2, aref_e2, H_e2;
  double cx, cy;               /* centroid of phi > 0 in the reference layer */
  int32_t flags;               /* SCD_CA_* */
  int32_t pad;
} scd_ca;                      /* angles in degrees, lengths in lattice units */

#define SCD_CA_NO_REF 1        /* phi <= 0 at the reference layer: E1 measured
                                  the base directly in the first fluid layer */
#define SCD_CA_E1_FLAT 2       /* E1 cap has no real base: reported as 180 */
#define SCD_CA_E2_FLAT 4       /* E2 likewise */
#define SCD_CA_RAY_LIMIT 8     /* a half-chord ray found no crossing in L/2 */
#define SCD_CA_NO_APEX 16      /* no crossing above the reference layer */
#define SCD_CA_NO_DROP 32      /* phi <= 0 on the first fluid node of the
                                  column: angles are NaN, ENOINTERFACE */
#define SCD_CA_E2_EMPTY 64     /* E2 column height <= 0 */
#define SCD_CA_E2_WHOLE_LAYER 128 /* phi <= 0 on the column at the reference
                                     layer: E2 summed the whole layer instead
                                     of the disk around the column */

typedef struct scd_lattice scd_lattice;

/* Bytes of one population buffer and of the work area for these params.
 * The work area holds link masks, reduction partials, observable scratch
 * and (with SCD_WITH_ADJOINT) the adjoint scratch. */
scd_status scd_sizes(const scd_params* p, size_t* pop_bytes, size_t* work_bytes);

/* Create a handle.  d_solid: N bytes, nonzero = wall node.  d_pop0, d_pop1:
 * the two population buffers (ping-pong); d_work: work area; all 256-byte
 * aligned device memory of the sizes given by scd_sizes.  stream: a
 * hipStream_t (NULL = default stream).  Validates the parameters (tau > 1/2,
 * rho_wall >= 0, g >= 0, dims >= 1) and writes *out. */
scd_status scd_create(const scd_params* p, const uint8_t* d_solid, void* d_pop0, void* d_pop1,
                      void* d_work, void* stream, scd_lattice** out);
scd_status scd_destroy(scd_lattice* h);

/* Change the physical parameters; dims, dtype and flags must not change. */
scd_status scd_set_params(scd_lattice* h, const scd_params* p);
scd_status scd_set_stream(scd_lattice* h, void* stream);

/* Sec. 2 initial state: C_k^a = zeta_k rho^a (fluid at rest) at fluid nodes,
 * from d_rho_a, d_rho_b (N doubles each).  Resets the step counter. */
scd_status scd_init_equilibrium(scd_lattice* h, const double* d_rho_a, const double* d_rho_b);

/* Advance nsteps >= 0 time steps of Eq. (LBeqs) (asynchronous). */
scd_status scd_step(scd_lattice* h, int64_t nsteps);
int64_t scd_step_count(const scd_lattice* h);

/* Plain <-> pop layout for a buffer of this handle's dims and dtype
 * (device to device, on the handle's stream; no synchronisation).  d_plain
 * holds 2 * 19 * N elements, d_blocked 2 * sp (padding slots of d_blocked
 * are left untouched by pack).  The two buffers must not overlap and must be
 * aligned to the element size; SCD_EINVAL otherwise. */
scd_status scd_pop_pack(const scd_lattice* h, const void* d_plain, void* d_blocked);
scd_status scd_pop_unpack(const scd_lattice* h, const void* d_blocked, void* d_plain);

/* Copy the current state out / in (pop layout, device to device). */
scd_status scd_get_state(scd_lattice* h, void* d_dst);
scd_status scd_set_state(scd_lattice* h, const void* d_src, int64_t step);

/* rho^a = sum_k C_k^a at fluid nodes, 0 at wall nodes; d_rho: 2 * N doubles */
scd_status scd_density(scd_lattice* h, double* d_rho);

/* Pressure tensor of Sec. 4.1 at every node, from the post-stream
 * populations of the current state.  At a fluid node
 *   P_ij = sum_a sum_k (c_ki - u_i)(c_kj - u_j) n_k^a
 *        + 1/2 sum_k W_k c_ki c_kj [psi^A G^A(y) psi^B(y) + psi^B G^B(y) psi^A(y)],
 * y = x + c_k, u = (sum_a j^a + F / 2) / sum_a rho^a the velocity of the
 * fluid (F the node's total Shan-Chen and wall force), G = g_ab at fluid and
 * g_wall^a at wall neighbours (whose psi is that of the wall content).  The
 * paper's 1/4 over the two ordered species pairs gives 1/2; its pair factor
 * is the dyad of x - x'.  At a wall node (the wall as a component of the
 * system) there is no kinetic part; the tensor is the wall's half of each
 * wall-fluid pair, 1/2 sum_{k: y fluid} W_k c_ki c_kj [g_wall^A psi^A(y)
 * psi_w^B + g_wall^B psi^B(y) psi_w^A].  d_P: caller-owned 6 * N doubles,
 * component-major d_P[c * N + i] with c = xx, yy, zz, xy, xz, yz.
 * Asynchronous on the handle's stream. */
scd_status scd_pressure_tensor(scd_lattice* h, double* d_P);

/* Surface tension integral of Eq. (gammaMechDef) for interfaces normal to z:
 * *h_gamma = sum over the planes z of the mean, over all nodes of the plane
 * (fluid and wall), of P_N - P_T = P_zz - (P_xx + P_yy) / 2.  A periodic box
 * with two interfaces holds twice the tension.  d_P: scratch of 6 * N
 * doubles (left holding the pressure tensor); h_profile: nz host doubles for
 * the plane means, or NULL.  Synchronises. */
scd_status scd_surface_tension_z(scd_lattice* h, double* d_P, double* h_gamma,
                                 double* h_profile);

/* Radial surface tension of Eq. (mechRadGamma) about h_center (3 host
 * doubles, lattice coordinates): shells of unit width, shell b holding the
 * fluid nodes with b <= |x - c| < b + 1 (minimum image on the periodic
 * axes, decided by exact comparisons on |x - c|^2), radius r_b = b + 1/2.
 * Per node P_N = d.P.d / |d|^2 and P_T = (tr P - P_N) / 2 with d = x - c
 * (the centre node adds 0).  h_profile / h_phi_profile (nbins host doubles
 * each, or NULL): shell means of P_N - P_T and of phi.  *h_Rs: first
 * outward crossing of the shell means of phi from > 0 to <= 0, linearly
 * interpolated; *h_gamma = sum over shells with r_b <= rmax of
 * (r_b / R_s)^2 profile[b].  d_P: scratch of 6 N doubles.  nbins in
 * [2, 1365].  Returns SCD_ENOINTERFACE (gamma, R_s NaN) without a
 * crossing.  Synchronises. */
scd_status scd_radial_tension(scd_lattice* h, double* d_P, const double* h_center, double rmax,
                              int32_t nbins, double* h_profile, double* h_phi_profile,
                              double* h_Rs, double* h_gamma);
/* The same with the minimum image taken only along the axes whose bit is set
 * in periodic (bit 0 x, bit 1 y, bit 2 z); along the others d is the plain
 * difference x - c.  scd_radial_tension is periodic = 7.  Use it for a
 * droplet between walls (a sessile droplet: periodic = 3), whose shells
 * must not wrap across the walls to the far side of the box.  periodic
 * outside [0, 7]: SCD_EINVAL. */
scd_status scd_radial_tension_axes(scd_lattice* h, double* d_P, const double* h_center,
                                   int32_t periodic, double rmax, int32_t nbins,
                                   double* h_profile, double* h_phi_profile, double* h_Rs,
                                   double* h_gamma);

/* Young's equation (Sec. 1, Eq. young) with the droplet species as the
 * liquid: theta = acos((gamma_SG - gamma_SL) / gamma_LG) in degrees, with
 * the cosine clamped to [-1, 1] (complete wetting 0, complete drying 180).
 * Host arithmetic only. */
double scd_young_angle(double gamma_sg, double gamma_sl, double gamma_lg);

/* Huang's a-priori estimate (Sec. 4.1, Eq. huangSigmaLG) for droplet
 * species A: cos(theta) = (G_ads,B - G_ads,A) / (g_ab (rho_in - rho_out) / 2)
 * with G_ads,a = g_wall^a psi(rho_wall^b), the repulsion species a feels from
 * the wall, and rho_in, rho_out the A densities of the A-rich and B-rich
 * bulk phases; degrees, clamped as above.  NaN if p is NULL. */
double scd_huang_angle(const scd_params* p, double rho_in, double rho_out);

/* Mass per species, total momentum and the all-finite flag, accumulated in
 * FP64 with a fixed reduction order (bit-reproducible).  Synchronises.
 * Returns SCD_ENONFINITE (with *out filled) if any population is not finite,
 * else SCD_EDRIFT (with *out filled) when the mass-drift watchdog is on and
 * either species' mass has drifted beyond its tolerance. */
scd_status scd_observables(scd_lattice* h, scd_obs* h_out);
/* Mass-drift watchdog (failure detection; the method conserves each
 * species' mass exactly, so any drift is rounding or a fault).  The
 * reference masses are those of the first scd_observables call after the
 * state was last set (scd_init_equilibrium, scd_set_state, scd_fill_state);
 * every later call measures (m_a - m_a,ref) / m_a,ref.  rel_tol 0 (the
 * default) only measures; rel_tol > 0 makes scd_observables return
 * SCD_EDRIFT when |drift| exceeds it for either species.  Setting the
 * tolerance keeps the reference.  Suggested tolerances: 1e-10 in FP64,
 * 1e-5 in FP32.  rel_tol < 0 or NaN: SCD_EINVAL. */
scd_status scd_set_mass_watchdog(scd_lattice* h, double rel_tol);
/* The relative drift of both species at the last scd_observables call
 * (h_drift: host array of 2; 0 at the call that took the reference). */
scd_status scd_mass_drift(const scd_lattice* h, double* h_drift);

/* Contact angle of the current state (Sec. 3), both estimators.
 * Synchronises.  Returns SCD_ENOINTERFACE with NaN angles and
 * SCD_CA_NO_DROP when phi <= 0 at the column's first fluid node. */
scd_status scd_contact_angle(scd_lattice* h, const scd_ca_cfg* cfg, scd_ca* h_out);

/* For callers that cannot allocate (code that must not call hipMalloc or an
 * allocating library routine: tight serving loops, harnesses that forbid
 * allocation): scd_contact_angle with its scratch (the phi layers and column,
 * the layer partials and the result slots) in a fixed device array of the
 * library instead of the lattice's work area.  The array holds planes of at
 * most 512 x 512 nodes and at most 4096 planes (4.1 MB per GPU, kept until
 * the process ends; each GPU has its own, looked up on the first call with
 * that GPU current); larger lattices get SCD_EUNSUPPORTED.  Same results,
 * flags and status as scd_contact_angle; synchronises.  Calls on one GPU
 * share the array: calls that overlap on one GPU (other threads or streams)
 * race and must be serialised by the caller. */
scd_status scd_contact_angle_static(scd_lattice* h, const scd_ca_cfg* cfg, scd_ca* h_out);

/* ---- adjoint (extension) ---- */
/* d_lambda (pop layout, dtype of the lattice) := dL/dC of the current state
 * for L = theta_E2 (radians) times dL_dtheta.  Synchronises. */
scd_status scd_ca_seed(scd_lattice* h, const scd_ca_cfg* cfg, double dL_dtheta, void* d_lambda);
/* One reverse step.  d_state_t: C^t (the state the forward step started
 * from); d_lam_in: lambda^{t+1} = dL/dC^{t+1}; d_lam_out: lambda^t (must not
 * alias d_lam_in).  With h_dparams != NULL: h_dparams[5] += dL/d{rho_wall_A,
 * rho_wall_B, g_ab, g_wall_A, g_wall_B} of this step, and the call
 * synchronises.  With h_dparams == NULL the step's gradient is added to a
 * device accumulator instead (no synchronisation); see scd_adjoint_reset /
 * scd_adjoint_read.  Needs SCD_WITH_ADJOINT. */
scd_status scd_adjoint_step(scd_lattice* h, const void* d_state_t, const void* d_lam_in,
                            void* d_lam_out, double* h_dparams);
/* Zero the device accumulator of the parameter gradient (asynchronous). */
scd_status scd_adjoint_reset(scd_lattice* h);
/* Copy the accumulator (5 doubles, same order) to the host.  Synchronises. */
scd_status scd_adjoint_read(scd_lattice* h, double* h_acc);

/* Checkpointed gradient of L = (theta_E2 - target_deg)^2 (deg^2) after
 * nsteps steps.  Forward: initialises from d_rho_a, d_rho_b (or, when both
 * are NULL, starts from the current state), runs nsteps storing the state
 * every ckpt_every steps into d_ckpt (ceil(nsteps / ckpt_every) population
 * buffers), then measures theta_E2: h_out[0] = loss, h_out[1] = theta_E2
 * (deg).  The parameters are constants of the run; the gradient is taken
 * over these nsteps steps only.
 * Backward (one level): for each segment in reverse, recomputes its states
 * into d_seg (scd_ckpt_seg_states buffers: ckpt_every - 1, or 2 when the
 * moment cache covers the segment; each recomputed step writes its slot
 * directly) and applies the adjoint steps; d_lam holds 2 population buffers
 * of scratch.  h_grad[5] = dL/d{rho_wall_A, rho_wall_B, g_ab, g_wall_A,
 * g_wall_B}.  Needs the state left by the forward call; on return the
 * lattice holds the first checkpoint (the state the forward call started
 * from).
 * Backward (two levels): inside each level-1 segment, recomputes level-2
 * checkpoints every K2 steps into d_mid (ceil(K1 / K2) buffers) and runs the
 * one-level sweep on each sub-segment with d_seg of scd_ckpt_seg_states(K2)
 * buffers: each step is recomputed twice and the memory is ceil(n/K1) +
 * ceil(K1/K2) + K2 + 1 states instead of ceil(n/K) + K + 1 (with the moment
 * cache: + 2 states + the cached moments, 8 x N reals per step of a
 * segment, instead of + K2 - 1 or K - 1 states). */
scd_status scd_ckpt_forward(scd_lattice* h, const double* d_rho_a, const double* d_rho_b,
                            int64_t nsteps, int64_t ckpt_every, void* d_ckpt,
                            const scd_ca_cfg* cfg, double target_deg, double* h_out);
/* Optional moment cache for the backward sweeps: d_buf holds nsteps blocks
 * of 8 x N reals (the lattice dtype: rho^A, rho^B, j^A (x, y, z), j^B (x, y,
 * z); caller-owned, kept alive while registered; nsteps = 0 unregisters).
 * When nsteps covers a recomputed segment (ckpt_every - 1 steps, or K2 - 1
 * with two levels) and the step variant is a multi-plane march (6, 7 or 8),
 * each recomputed step also writes the densities and momenta of the
 * post-stream populations of the state it reads, and the adjoint of that
 * state uses them instead of pulling its populations to form them.  These
 * are the same sums in the same order, so the gradient is the same bit for
 * bit.  Such an adjoint reads nothing else of its state, so the recomputed
 * states then alternate between two buffers of d_seg. */
scd_status scd_ckpt_moment_cache(scd_lattice* h, void* d_buf, int64_t nsteps);
/* Population buffers d_seg must hold for segments of seg_len steps with the
 * lattice's current step variant and moment cache: 2 (at most seg_len - 1)
 * when the cache covers the segment, else seg_len - 1 (0 for seg_len 1). */
scd_status scd_ckpt_seg_states(const scd_lattice* h, int64_t seg_len, int64_t* h_states);
scd_status scd_ckpt_backward(scd_lattice* h, int64_t nsteps, int64_t ckpt_every,
                             const void* d_ckpt, void* d_seg, void* d_lam,
                             const scd_ca_cfg* cfg, double target_deg, double* h_grad);
scd_status scd_ckpt_backward2(scd_lattice* h, int64_t nsteps, int64_t K1, int64_t K2,
                              const void* d_ckpt, void* d_mid, void* d_seg, void* d_lam,
                              const scd_ca_cfg* cfg, double target_deg, double* h_grad);

/* ---- launch control (extension) ---- */
/* The fused step is compiled in several variants: a tile of tx * ty node
 * columns marched along z, a z-march variant and a minimum number of waves
 * per SIMD.  z-march variants: 0 one thread per node, populations kept in
 * registers; 1 the same, pulled again from cache at the collision; 2 two
 * threads per node (one per species); 3 as 2 with streaming stores; 4 as 3,
 * software-pipelined; 5 as 3 with all loads of a plane issued together;
 * 6, 7, 8 as 5 with two, three or four planes per barrier.  scd_tile_list
 * writes up to cap rows (tx, ty, z-march variant, waves) into h_rows (4
 * int32 per row) and the number of variants into *n.  A lattice uses one
 * variant index and a z-chunk of zc planes per workgroup; the default is
 * variant 7 (32 x 4, one wave) in FP64 and 6 (64 x 4, two waves) in FP32,
 * with zc from a model of workgroup rounds. */
scd_status scd_tile_list(int32_t* h_rows, int32_t cap, int32_t* n);
scd_status scd_tile_set(scd_lattice* h, int32_t variant, int32_t zc);
scd_status scd_tile_get(const scd_lattice* h, int32_t* variant, int32_t* zc);
/* Time every compiled variant with several z-chunks (4, 8, ..., 128 and the
 * chunk the default wave-count model picks for that variant) on this
 * lattice and keep the fastest: h_best[2] = variant, zc; *h_ms = its time
 * per step.  The
 * trial steps advance (and overwrite) the lattice state: re-initialise it
 * afterwards.  cache_path (may be NULL): JSON-lines file of earlier results
 * keyed by dims, dtype, device and variant count; a hit skips the trials. */
scd_status scd_autotune(scd_lattice* h, int32_t steps_per_trial, const char* cache_path,
                        int32_t* h_best, double* h_ms);

/* Capture nsteps (even, > 0) steps into a HIP graph on the handle's stream,
 * then replay it; scd_graph_replay advances the state by reps * nsteps. */
scd_status scd_graph_capture(scd_lattice* h, int64_t nsteps);
scd_status scd_graph_replay(scd_lattice* h, int64_t reps);

/* ---- batched launch (extension) ----
 * n lattices of any sizes (one dtype) advance together: a step is one
 * launch per group of members (members of one step variant, at most 16 per
 * launch, whose descriptors travel in the kernel arguments), whose
 * workgroups walk the members' (tile column, z-chunk) items; a group of one
 * member with one workgroup per item is launched as scd_step launches it.  The caller provides one
 * device arena of scd_batch_sizes bytes that holds every lattice's two
 * population buffers and work area and the work list.  d_solid: host array
 * of n device pointers to the solid masks (kept alive by the caller). */
typedef struct scd_batch scd_batch;
scd_status scd_batch_sizes(int32_t n, const scd_params* p, size_t* arena_bytes);
scd_status scd_batch_create(int32_t n, const scd_params* p, const uint8_t* const* d_solid,
                            void* d_arena, void* stream, scd_batch** out);
scd_status scd_batch_destroy(scd_batch* b);
/* A lattice handle that views member i (observables, contact angle,
 * density, state copies); owned by the batch, do not destroy or step it. */
scd_status scd_batch_lattice(scd_batch* b, int32_t i, scd_lattice** view);
scd_status scd_batch_init_equilibrium(scd_batch* b, int32_t i, const double* d_rho_a,
                                      const double* d_rho_b);
/* Step variant (see scd_tile_list), z-chunk (1 .. 32767 planes, else
 * SCD_EINVAL) and number of persistent workgroups (grid), the same for every
 * member; grid 0 (the default) launches one workgroup per (lattice, tile)
 * item, a shorter grid walks the items persistently (rounded up to a
 * multiple of 8).  Items are dealt to the 8 XCDs in contiguous ranges (the
 * chunks of a tile column and the columns of a lattice stay on one XCD), and
 * neighbouring z-chunks march in opposite directions, as in scd_step.
 * Defaults: the single-lattice default variant of the dtype, 32-plane
 * chunks, grid 0. */
scd_status scd_batch_set_tile(scd_batch* b, int32_t variant, int32_t zc, int32_t grid);
/* Variant and z-chunk of member i alone (the grid stays).  Members are
 * stepped in groups of equal variant, one launch per group and step, each
 * group's items dealt to the XCDs as above. */
scd_status scd_batch_set_member_tile(scd_batch* b, int32_t i, int32_t variant, int32_t zc);
scd_status scd_batch_member_tile(const scd_batch* b, int32_t i, int32_t* variant, int32_t* zc);
/* Cache blocking across members: the members are packed, in index order,
 * into sets whose state (both population buffers and the link masks) stays
 * within set_bytes (a member larger than that forms a set alone), and
 * scd_batch_step, like a captured graph, runs every step of a call on one
 * set before it moves to the next.  A set's state then stays in the 256 MB
 * last-level cache (MALL) between its steps instead of being evicted by the
 * other members' traffic.  The members are independent, so the result is
 * the same for any set_bytes.  0 (the default) makes one set of all members,
 * which advance one step per launch.  set_bytes < 0: SCD_EINVAL.  Drops a
 * captured graph.  scd_batch_blocking returns the setting and the number of
 * sets it gives. */
scd_status scd_batch_set_blocking(scd_batch* b, int64_t set_bytes);
scd_status scd_batch_blocking(const scd_batch* b, int64_t* set_bytes, int32_t* nsets);
scd_status scd_batch_step(scd_batch* b, int64_t nsteps);
scd_status scd_batch_graph_capture(scd_batch* b, int64_t nsteps);
scd_status scd_batch_graph_replay(scd_batch* b, int64_t reps);
/* Pick the batch's tiles and cache blocking by timing: (1) every compiled
 * variant for all members at 16- and 32-plane chunks, one workgroup per
 * item, one set; (2) for each member the variant and z-chunk that step it
 * alone fastest (each variant at the wave-count model's chunk for that
 * lattice and at 4, 8, 16, 32 and 64 planes), then those tiles, and those
 * variants at each member's model chunk or one chunk of {8, 16, 32, 48, 64}
 * for all, x grid {one workgroup per item, 4 per compute unit}; (3) sets of
 * at most 64, 128, 192 or 256 MiB, or one member per set, with the best so
 * far and with the per-member tiles; the fastest of all is kept.  A trial
 * is steps_per_trial steps (plus one warm-up) per set; h_best = {the most common member variant, zc
 * (0 when the members' chunks differ), grid}, h_ms its time per step.  The
 * members advance by every trial step (re-initialise afterwards for a clean
 * start).  cache_path (or NULL): JSON-lines file; a line with the same key
 * (member shapes, dtype, device, variant count) and its member variants,
 * chunks and set budget is used without timing, a new result is appended.
 * Drops a captured graph. */
scd_status scd_batch_autotune(scd_batch* b, int32_t steps_per_trial, const char* cache_path,
                              int32_t* h_best, double* h_ms);

/* Fill each of the 38 * N entries of the current state with value
 * (for tests of the observables) */
scd_status scd_fill_state(scd_lattice* h, double value);

/* Measurement helper: copy bytes (a multiple of 8) from d_src to d_dst
 * (device, 8-byte aligned, not overlapping) with a plain grid-stride copy
 * kernel on the stream (may be NULL for the default stream); asynchronous.
 * Timed by the caller, it gives the attainable HBM rate of a read-once
 * write-once sweep: the ceiling the fused step's rate is compared with. */
scd_status scd_stream_copy(const void* d_src, void* d_dst, size_t bytes, void* stream);
/* Measurement helper: the fused step's data movement without its
 * arithmetic.  One launch on the handle's stream in which every fluid node
 * pulls its 2 x 19 populations from the current state exactly as a step does
 * (periodic neighbours, mid-grid bounce-back) and writes them unchanged to
 * the other population buffer.  The current state is left as it is; the
 * other buffer (the next step's destination) is overwritten.  Timed by the
 * caller, it gives the HBM rate the state layout allows, the ceiling the
 * step's rate is compared with.  Asynchronous. */
scd_status scd_pull_copy(scd_lattice* h);

const char* scd_last_error(void);
const char* scd_version(void);

#ifdef __cplusplus
}
#endif
#endif
