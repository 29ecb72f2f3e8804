// adjoint.hip -- reverse-mode step of the fused lattice update (extension:
// the exact transpose of every sub-step of Sec. 2, applied in reverse order).
//
// Given the state C^t and lambda' = dL/dC^{t+1}, one reverse step produces
// lambda = dL/dC^t and the gradient with respect to the wall contents, the
// fluid coupling and the wall couplings.  Two passes over the lattice (three
// in FP32), after the post-stream densities of C^t (computed or cached):
//   1. per fluid node: recompute the forward quantities (pull, moments, psi,
//      force from the neighbours' post-stream densities, velocities) and
//      transpose the collision (Eq. Equil), the velocity shift and the local
//      part of the force; store q^a = psi^a dL/dF^a, D^a = dL/drho^a and
//      the vector e = dL/du' / R, from which dL/dj^a = e / tau^a, and
//      accumulate the gradient of the wall parameters;
//   2. per node: add the transposed force stencil, i.e. the gather
//      -g_ab sum_k W_k q^b(y - c_k) . c_k, through psi'(rho) to D, with the
//      same gather giving the g_ab gradient
//      (-psi^b(y) times it, summed), then stream transposed with
//      bounce-back, as a push of
//      dL/dn_k = D + (e / tau) . c_k + (1 - 1/tau) lambda'_k to x - c_k (or
//      to the node itself on the opposite velocity next to a wall).
#include "common.hpp"
#include "kernels.hpp"

namespace scd {

template <int NV>
__device__ __forceinline__ void block_sum_adj(double (&v)[NV], double* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int j = 0; j < NV; ++j)
    for (int off = 32; off > 0; off >>= 1) v[j] += __shfl_xor(v[j], off, 64);
  if (lane == 0)
    for (int j = 0; j < NV; ++j) sh[j * 16 + wave] = v[j];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int j = 0; j < NV; ++j) {
      double s = 0;
      for (int w = 0; w < nw; ++w) s += sh[j * 16 + w];
      v[j] = s;
    }
}

// pair_moment below takes velocity k + 1 as the opposite of k for odd k.
constexpr bool opposite_pairs_adjacent() {
  for (int k = 1; k < Q; k += 2)
    if (OPP[k] != k + 1 || CX[k + 1] != -CX[k] || CY[k + 1] != -CY[k] || CZ[k + 1] != -CZ[k])
      return false;
  return true;
}
static_assert(opposite_pairs_adjacent(), "velocity k + 1 must be the opposite of odd k");

// psi (and psi') of densities with the form tested once, outside any loop:
// written as one select per value, the exponential of the other form is
// evaluated for every value whichever form is in use.
template <typename real, int NV>
__device__ __forceinline__ void psi_in_place(int form, real (&v)[NV], int k0) {
  if (form == 1) {
#pragma unroll
    for (int k = k0; k < NV; ++k) v[k] = real(1) - exp(-v[k]);
  }
}
template <typename real>
__device__ __forceinline__ void psi_pair(int form, real rho, real& psi, real& dpsi) {
  if (form == 1) {
    const real t = exp(-rho);
    psi = real(1) - t;
    dpsi = t;
  } else {
    psi = rho;
    dpsi = real(1);
  }
}

// dL/drho and dL/du of the equilibrium term n^eq_k(rho, u) / tau of one
// species' collision (Eq. Equil, cubic in u), given lambda' of its 19
// populations.  With G_k = W_k lambda'_k, s_k = c_k . u, a = 3 - 9/2 u.u and
// b = 1 - 3/2 u.u:
//   tau dL/drho = sum_k G_k (b + s_k (a + s_k (9/2 + 9/2 s_k))),
//   tau dL/du_d = rho [sum_k G_k c_kd (a + s_k (9 + 27/2 s_k)) - m u_d],
//   m = sum_k G_k (3 + 9 s_k),
// taking s_k and the c_kd terms only along the components c_k moves in
// (c_kd = +-1 or 0).  The velocity sums start at -0, which the first
// addition leaves exactly.  The velocities are taken one at a time, so that
// each lambda'_k is released once used.
template <typename real>
__device__ __forceinline__ void equil_adj(const real (&lm)[Q], real inv_tau, real rho,
                                          const real (&u)[3], real& drho, real (&du)[3]) {
  const real uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const real a = real(3) - real(4.5) * uu, b = real(1) - real(1.5) * uu;
  const real G0 = real(WEIGHT[0]) * lm[0];
  real dr = G0 * b, m = real(3) * G0;
  real v[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) v[d] = real(-0.0);
#pragma unroll
  for (int k = 1; k < Q; ++k) {
    const int c[3] = {CX[k], CY[k], CZ[k]};
    const real G = real(WEIGHT[k]) * lm[k];
    real s = real(-0.0);
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (c[d]) s += c[d] > 0 ? u[d] : -u[d];
    dr += G * (b + s * (a + s * (real(4.5) + real(4.5) * s)));
    m += G * (real(3) + real(9) * s);
    const real w = G * (a + s * (real(9) + real(13.5) * s));
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (c[d]) v[d] += c[d] > 0 ? w : -w;
  }
  drho = dr * inv_tau;
  const real rt = rho * inv_tau;
#pragma unroll
  for (int d = 0; d < 3; ++d) du[d] = rt * (v[d] - m * u[d]);
}

// v = sum over the 18 moving velocities of e_k c_k, taken over the opposite
// pairs as (e_k - e_{k+1}) c_k along the components c_k moves in.
template <typename real>
__device__ __forceinline__ void pair_moment(const real (&e)[Q], real (&v)[3]) {
  v[0] = v[1] = v[2] = real(-0.0);
#pragma unroll
  for (int k = 1; k < Q; k += 2) {
    const int c[3] = {CX[k], CY[k], CZ[k]};
    const real t = e[k] - e[k + 1];
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (c[d]) v[d] += c[d] > 0 ? t : -t;
  }
}

// Post-stream densities and momenta of the state a reverse step reads:
// rho[a N + i] and jm[(3 a + d) N + i], zero at wall nodes.  These are the
// sums of the pulled populations in the order of moments(), the same values
// the forward step forms, so the reverse step built on them is exact.
template <typename real>
__global__ __launch_bounds__(256) void k_stream_moments(const real* __restrict__ C,
                                                        const uint32_t* __restrict__ links,
                                                        real* __restrict__ rho,
                                                        real* __restrict__ jm, int nx, int ny,
                                                        int nz) {
  const int N = nx * ny * nz;
  const PopGeo pg = pop_geo(nx, ny, nz);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    const uint32_t lb = links[i];
    real r[2] = {0, 0}, j[2][3] = {{0, 0, 0}, {0, 0, 0}};
    if (!(lb & SELF_SOLID)) {
      int xs[3], ys[3], zs[3];
      axis3(i % nx, nx, xs);
      axis3((i / nx) % ny, ny, ys);
      axis3(i / (nx * ny), nz, zs);
      real n[38];
      pull38(C, pg, xs, ys, zs, nx, lb, n);  // 32-bit byte offsets, as the step's pulls
      moments(&n[0], r[0], j[0][0], j[0][1], j[0][2]);
      moments(&n[Q], r[1], j[1][0], j[1][1], j[1][2]);
    }
    rho[i] = r[0];
    rho[(size_t)N + i] = r[1];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int d = 0; d < 3; ++d) jm[(size_t)(3 * a + d) * N + i] = j[a][d];
  }
}

// Local part of the reverse step at every node.  rho comes from rhof and j
// from jm (3 fields per species), both filled beforehand: by
// k_stream_moments, or by a recomputed forward step of a checkpointed sweep
// (its 8 stored fields: rho^A, rho^B, j^A, j^B); no population is pulled.
template <typename real>
__global__ __launch_bounds__(256) void k_adj_local(const real* __restrict__ jm,
                                                   const real* __restrict__ lam,
                                                   const uint32_t* __restrict__ links,
                                                   const real* __restrict__ rhof, int nx, int ny,
                                                   int nz, Phys<real> ph, real* __restrict__ qf,
                                                   real* __restrict__ df, real* __restrict__ ef,
                                                   double* __restrict__ partials, int accumulate) {
  __shared__ double sh[5 * 16];
  const int N = nx * ny * nz;
  const PopGeo pg = pop_geo(nx, ny, nz);
  const int stride = gridDim.x * blockDim.x;
  double gp[5] = {0, 0, 0, 0, 0};  // rho_wall_A, rho_wall_B, g_ab, g_wall_A, g_wall_B
  // neighbour densities and lambda' are read at a uniform base plus a 32-bit
  // byte offset (a field of N reals and a species of lambda stay below 4 GiB)
  constexpr uint32_t SZ = sizeof(real);
  const char* __restrict__ rbase[2] = {reinterpret_cast<const char*>(rhof),
                                       reinterpret_cast<const char*>(rhof + N)};
  const char* __restrict__ lbase[2] = {reinterpret_cast<const char*>(lam),
                                       reinterpret_cast<const char*>(lam + pg.sp)};
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
    const uint32_t lb = links[i];
    if (lb & SELF_SOLID) {
      for (int c = 0; c < 6; ++c) qf[(size_t)c * N + i] = 0;
      for (int d = 0; d < 3; ++d) ef[(size_t)d * N + i] = 0;
      df[i] = 0;
      df[(size_t)N + i] = 0;
      continue;
    }
    int xs[3], ys[3], zs[3];
    axis3(i % nx, nx, xs);
    axis3((i / nx) % ny, ny, ys);
    axis3(i / (nx * ny), nz, zs);
    const uint32_t si = pop_slot(pg, zs[1], ys[1] * nx + xs[1]);
    real rho[2], j[2][3];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      rho[a] = rhof[(size_t)a * N + i];
#pragma unroll
      for (int d = 0; d < 3; ++d) j[a][d] = jm[(size_t)(3 * a + d) * N + i];
    }
    real psi[2], dpsi[2];
    psi_pair(ph.psi_form, rho[0], psi[0], dpsi[0]);
    psi_pair(ph.psi_form, rho[1], psi[1], dpsi[1]);
    // lambda' of both species, requested before the neighbour densities so
    // that all 74 loads of the node are in flight together
    real lm[2][Q];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int k = 0; k < Q; ++k) lm[a][k] = ld_off<real>(lbase[a], (si + (uint32_t)k * PBLK) * SZ);
    // S^a = sum_k W_k G^a(y) psi^b(y) c_k over the 18 neighbours y = x + c_k,
    // and Wv = sum over the wall neighbours of W_k c_k (for the gradient of
    // the wall parameters).  Every neighbour's densities are loaded (a wall
    // node's field entry is a valid zero) and the wall content selected
    // afterwards, so the loads carry no branch between them.
    real nA[Q], nB[Q];
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      const uint32_t yo = (uint32_t)nbr_index(xs, ys, zs, nx, ny, CX[k], CY[k], CZ[k]) * SZ;
      nA[k] = ld_off<real>(rbase[0], yo);
      nB[k] = ld_off<real>(rbase[1], yo);
    }
    psi_in_place(ph.psi_form, nA, 1);  // now psi^A and psi^B of the neighbours
    psi_in_place(ph.psi_form, nB, 1);
    real eA[Q], eB[Q], wv[Q];
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      const bool wall = (lb >> k) & 1u;
      const real w = (CX[k] * CX[k] + CY[k] * CY[k] + CZ[k] * CZ[k]) == 1 ? ph.wa : ph.wd;
      eA[k] = wall ? w * ph.gw[0] * ph.psiw[1] : w * ph.gab * nB[k];
      eB[k] = wall ? w * ph.gw[1] * ph.psiw[0] : w * ph.gab * nA[k];
      wv[k] = wall ? w : real(0);
    }
    real S[2][3], Wv[3];
    pair_moment(eA, S[0]);
    pair_moment(eB, S[1]);
    pair_moment(wv, Wv);
    real F[2][3];
    for (int a = 0; a < 2; ++a)
      for (int d = 0; d < 3; ++d) F[a][d] = -psi[a] * S[a][d];
    // three reciprocals serve every quotient below
    const real Rt = rho[0] * ph.inv_tau[0] + rho[1] * ph.inv_tau[1];
    const real iRt = real(1) / Rt;
    const real ir[2] = {real(1) / rho[0], real(1) / rho[1]};
    const real tr[2] = {ph.tau[0] * ir[0], ph.tau[1] * ir[1]};  // tau^a / rho^a
    real up[3], u[2][3];
    for (int d = 0; d < 3; ++d) up[d] = (j[0][d] * ph.inv_tau[0] + j[1][d] * ph.inv_tau[1]) * iRt;
    for (int a = 0; a < 2; ++a)
      for (int d = 0; d < 3; ++d) u[a][d] = up[d] + tr[a] * F[a][d];

    // transpose of the collision C' = n (1 - 1/tau) + n^eq(rho, u) / tau
    real drho[2], du[2][3];
#pragma unroll
    for (int a = 0; a < 2; ++a) equil_adj(lm[a], ph.inv_tau[a], rho[a], u[a], drho[a], du[a]);
    // transpose of u^a = u' + tau^a F^a / rho^a, u' = J / R
    real dF[2][3], dup[3] = {0, 0, 0};
    for (int a = 0; a < 2; ++a) {
      real Fdu = 0;
      for (int d = 0; d < 3; ++d) {
        dF[a][d] = tr[a] * du[a][d];
        Fdu += F[a][d] * du[a][d];
        dup[d] += du[a][d];
      }
      drho[a] += -tr[a] * Fdu * ir[a];
    }
    const real dupu = dup[0] * up[0] + dup[1] * up[1] + dup[2] * up[2];
    // dL/dj^a = dup / (tau^a R): one vector serves both species
    for (int d = 0; d < 3; ++d) ef[(size_t)d * N + i] = dup[d] * iRt;
    for (int a = 0; a < 2; ++a) drho[a] += -dupu * (ph.inv_tau[a] * iRt);
    // transpose of the force: local part and the gradient of the wall
    // parameters (the fluid neighbours' part, the g_ab gradient, is taken in
    // the transposed stencil, which gathers the same pair products)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int b = 1 - a;
      const real dpsi_self = -(dF[a][0] * S[a][0] + dF[a][1] * S[a][1] + dF[a][2] * S[a][2]);
      for (int d = 0; d < 3; ++d) qf[(size_t)(a * 3 + d) * N + i] = psi[a] * dF[a][d];
      df[(size_t)a * N + i] = drho[a] + dpsi[a] * dpsi_self;
      // sum over the wall neighbours of -psi^a W_k dF^a . c_k
      const double t = (double)(-psi[a] * (dF[a][0] * Wv[0] + dF[a][1] * Wv[1] + dF[a][2] * Wv[2]));
      gp[3 + a] += (double)ph.psiw[b] * t;
      gp[b] += (double)ph.gw[a] * t * (double)ph.dpsiw[b];
    }
  }
  block_sum_adj<5>(gp, sh);
  // a block owns its slot, so accumulating over steps is deterministic
  if (threadIdx.x == 0)
    for (int c = 0; c < 5; ++c)
      partials[blockIdx.x * RED_STRIDE + c] =
          accumulate ? partials[blockIdx.x * RED_STRIDE + c] + gp[c] : gp[c];
}

// The same local pass with the two species of a node on the two halves of
// a wave: lanes 0-31 take species A of 32 consecutive nodes, lanes 32-63
// species B of the same nodes, and the partners exchange the few values
// that couple the species (the other species' density and momentum, and its
// velocity adjoint) through __shfl_xor(., 32).  A lane then holds lambda' of
// one species and the neighbour densities of the other (the force on
// species a is built from psi^b of the neighbours), half the registers of
// the pass above, so that the FP64 pass runs at two waves per SIMD instead
// of one.  The arithmetic of every node and species is the same, in the
// same order; only the wall-parameter partials are summed in another order.
template <typename real>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_adj_local_split(
    const real* __restrict__ jm, const real* __restrict__ lam, const uint32_t* __restrict__ links,
    const real* __restrict__ rhof, int nx, int ny, int nz, Phys<real> ph, real* __restrict__ qf,
    real* __restrict__ df, real* __restrict__ ef, double* __restrict__ partials, int accumulate) {
  __shared__ double sh[5 * 16];
  const int N = nx * ny * nz;
  const PopGeo pg = pop_geo(nx, ny, nz);
  const int lane = threadIdx.x & 63;
  const int a = lane >> 5, b = 1 - a;
  const int waves = (gridDim.x * blockDim.x) >> 6;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  double gp[5] = {0, 0, 0, 0, 0};  // rho_wall_A, rho_wall_B, g_ab, g_wall_A, g_wall_B
  constexpr uint32_t SZ = sizeof(real);
  const char* __restrict__ rother = reinterpret_cast<const char*>(rhof + (size_t)b * N);
  const char* __restrict__ lown = reinterpret_cast<const char*>(lam + (size_t)a * pg.sp);
  // every lane of a wave runs the same number of iterations, so that the
  // partners of a node are always active together
  for (int base = wave * 32; base < N; base += waves * 32) {
    const int i = base + (lane & 31);
    const bool in = i < N;
    const uint32_t lb = in ? links[i] : SELF_SOLID;
    const bool fluid = !(lb & SELF_SOLID);
    int xs[3], ys[3], zs[3];
    const int ic = in ? i : 0;
    axis3(ic % nx, nx, xs);
    axis3((ic / nx) % ny, ny, ys);
    axis3(ic / (nx * ny), nz, zs);
    const uint32_t si = pop_slot(pg, zs[1], ys[1] * nx + xs[1]);
    // own species' moments and lambda'; the other species' neighbour
    // densities (a wall neighbour's entry is a valid zero, its wall content
    // is selected below)
    real rho_s = 0, js[3] = {0, 0, 0};
    real lm[Q], nb[Q];
    if (fluid) {
      rho_s = rhof[(size_t)a * N + i];
#pragma unroll
      for (int d = 0; d < 3; ++d) js[d] = jm[(size_t)(3 * a + d) * N + i];
#pragma unroll
      for (int k = 0; k < Q; ++k) lm[k] = ld_off<real>(lown, (si + (uint32_t)k * PBLK) * SZ);
#pragma unroll
      for (int k = 1; k < Q; ++k)
        nb[k] = ld_off<real>(rother, (uint32_t)nbr_index(xs, ys, zs, nx, ny, CX[k], CY[k], CZ[k]) * SZ);
    }
    // the partner's density and momentum (both lanes of a node take part)
    const real rho_o = __shfl_xor(rho_s, 32, 64);
    const real jo0 = __shfl_xor(js[0], 32, 64), jo1 = __shfl_xor(js[1], 32, 64),
               jo2 = __shfl_xor(js[2], 32, 64);
    real rho[2], j[2][3];
    rho[a] = rho_s;
    rho[b] = rho_o;
    j[a][0] = js[0]; j[a][1] = js[1]; j[a][2] = js[2];
    j[b][0] = jo0; j[b][1] = jo1; j[b][2] = jo2;
    // S^a = sum_k W_k G^a(y) psi^b(y) c_k and Wv = sum over the wall
    // neighbours of W_k c_k
    real S[3] = {0, 0, 0}, Wv[3] = {0, 0, 0};
    if (fluid) {
      psi_in_place(ph.psi_form, nb, 1);  // now psi^b of the neighbours
      real e[Q], wv[Q];
#pragma unroll
      for (int k = 1; k < Q; ++k) {
        const bool wall = (lb >> k) & 1u;
        const real w = (CX[k] * CX[k] + CY[k] * CY[k] + CZ[k] * CZ[k]) == 1 ? ph.wa : ph.wd;
        e[k] = wall ? w * ph.gw[a] * ph.psiw[b] : w * ph.gab * nb[k];
        wv[k] = wall ? w : real(0);
      }
      pair_moment(e, S);
      pair_moment(wv, Wv);
    }
    real psi_s, dpsi_s;
    psi_pair(ph.psi_form, rho[a], psi_s, dpsi_s);
    real F[3];
    for (int d = 0; d < 3; ++d) F[d] = -psi_s * S[d];
    // two reciprocals serve every quotient below
    const real Rt = rho[0] * ph.inv_tau[0] + rho[1] * ph.inv_tau[1];
    const real iRt = real(1) / Rt, ir = real(1) / rho[a];
    const real tr = ph.tau[a] * ir;  // tau^a / rho^a
    real up[3], u[3];
    for (int d = 0; d < 3; ++d) up[d] = (j[0][d] * ph.inv_tau[0] + j[1][d] * ph.inv_tau[1]) * iRt;
    for (int d = 0; d < 3; ++d) u[d] = up[d] + tr * F[d];

    // transpose of the collision of species a
    real drho = 0, du[3] = {0, 0, 0};
    if (fluid) {
      // the terms of equil_adj in their first form, one velocity at a time
      // (the moment form needs more registers than two waves per SIMD
      // leave this kernel)
      const real uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        const int c[3] = {CX[k], CY[k], CZ[k]};
        const real g = lm[k] * ph.inv_tau[a];
        real s = real(-0.0);
#pragma unroll
        for (int d = 0; d < 3; ++d)
          if (c[d]) s += c[d] > 0 ? u[d] : -u[d];
        const real P = real(1) + real(3) * s + real(4.5) * s * s - real(1.5) * uu +
                       real(4.5) * s * s * s - real(4.5) * uu * s;
        const real Ps = real(3) + real(9) * s + real(13.5) * s * s - real(4.5) * uu;
        const real Pq = real(-1.5) - real(4.5) * s;
        const real wg = real(WEIGHT[k]) * g;
        drho += wg * P;
        const real wr = wg * rho[a];
#pragma unroll
        for (int d = 0; d < 3; ++d)
          du[d] += wr * ((c[d] ? (c[d] > 0 ? Ps : -Ps) : real(-0.0)) + real(2) * Pq * u[d]);
      }
    }
    // transpose of u^a = u' + tau^a F^a / rho^a, u' = J / R; dup sums the
    // velocity adjoints of both species, in species order
    real dF[3], Fdu = 0;
    for (int d = 0; d < 3; ++d) {
      dF[d] = tr * du[d];
      Fdu += F[d] * du[d];
    }
    drho += -tr * Fdu * ir;
    const real duo0 = __shfl_xor(du[0], 32, 64), duo1 = __shfl_xor(du[1], 32, 64),
               duo2 = __shfl_xor(du[2], 32, 64);
    const real duA[3] = {a ? duo0 : du[0], a ? duo1 : du[1], a ? duo2 : du[2]};
    const real duB[3] = {a ? du[0] : duo0, a ? du[1] : duo1, a ? du[2] : duo2};
    real dup[3];
    for (int d = 0; d < 3; ++d) {
      dup[d] = 0;
      dup[d] += duA[d];
      dup[d] += duB[d];
    }
    if (!in) continue;
    if (!fluid) {
      for (int d = 0; d < 3; ++d) qf[(size_t)(a * 3 + d) * N + i] = 0;
      ef[(size_t)a * N + i] = 0;
      if (a == 0) ef[2 * (size_t)N + i] = 0;
      df[(size_t)a * N + i] = 0;
      continue;
    }
    const real dupu = dup[0] * up[0] + dup[1] * up[1] + dup[2] * up[2];
    // dL/dj^a = dup / (tau^a R): one vector for both species, its
    // components x and y stored by the lanes of species A and B, z by A
    ef[(size_t)a * N + i] = (a ? dup[1] : dup[0]) * iRt;
    if (a == 0) ef[2 * (size_t)N + i] = dup[2] * iRt;
    drho += -dupu * (ph.inv_tau[a] * iRt);
    // transpose of the force: local part and the gradient of the wall
    // parameters (the fluid neighbours' part, the g_ab gradient, is taken in
    // the transposed stencil)
    const real dpsi_self = -(dF[0] * S[0] + dF[1] * S[1] + dF[2] * S[2]);
    for (int d = 0; d < 3; ++d) qf[(size_t)(a * 3 + d) * N + i] = psi_s * dF[d];
    df[(size_t)a * N + i] = drho + dpsi_s * dpsi_self;
    const double t = (double)(-psi_s * (dF[0] * Wv[0] + dF[1] * Wv[1] + dF[2] * Wv[2]));
    gp[3 + a] += (double)ph.psiw[b] * t;
    gp[b] += (double)ph.gw[a] * t * (double)ph.dpsiw[b];
  }
  block_sum_adj<5>(gp, sh);
  if (threadIdx.x == 0)
    for (int c = 0; c < 5; ++c)
      partials[blockIdx.x * RED_STRIDE + c] =
          accumulate ? partials[blockIdx.x * RED_STRIDE + c] + gp[c] : gp[c];
}

// The gather of the transposed force stencil at fluid node y:
// acc[b] = sum_k W_k q^a(y - c_k) . c_k, a != b, which adds
// psi'(rho^b(y)) * (-g_ab acc[b]) to D^b(y)
template <typename real>
__device__ __forceinline__ void stencil_acc(const real* __restrict__ qf, int N,
                                            const int (&xs)[3], const int (&ys)[3],
                                            const int (&zs)[3], int nx, int ny,
                                            const Phys<real>& ph, real (&acc)[2]) {
  acc[0] = acc[1] = 0;  // acc[b] from q of the other species
#pragma unroll
  for (int k = 1; k < Q; ++k) {
    const int x = nbr_index(xs, ys, zs, nx, ny, -CX[k], -CY[k], -CZ[k]);
    const real w = (CX[k] * CX[k] + CY[k] * CY[k] + CZ[k] * CZ[k]) == 1 ? ph.wa : ph.wd;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      // only the components along which c_k moves (60 of the 108 loads)
      real qc = 0;
      if (CX[k]) qc += qf[(size_t)(a * 3 + 0) * N + x] * CX[k];
      if (CY[k]) qc += qf[(size_t)(a * 3 + 1) * N + x] * CY[k];
      if (CZ[k]) qc += qf[(size_t)(a * 3 + 2) * N + x] * CZ[k];
      acc[1 - a] += w * qc;
    }
  }
}

// The g_ab part of the parameter gradient, gathered with the stencil: the
// local pass would add -psi^a(x) W_k dF^a(x) . c_k psi^b(y) for every fluid
// pair (x, y = x + c_k); summed at y this is -psi^b(y) acc[b](y).  Each
// workgroup writes (or, accumulating, adds) its sum to column GAB_COL of its
// partials row.
constexpr int GAB_COL = 5;

// Transposed streaming with the transposed force stencil in the same pass.
// First the non-local part of dL/drho at fluid node y,
// from q of the other species at the 18 upstream nodes:
//   D^a(y) = D_local^a(y) + psi'(rho^a(y)) * (-g_ab sum_k W_k q^b(y - c_k) . c_k)
// (only the components along which c_k moves are loaded: 60 loads).  Then
// the push: mu_k(y) = D(y) + e(y) . c_k / tau + (1 - 1/tau) lambda'_k(y)
// (= dL/dn_k(y)) goes to lambda_k(y - c_k) when y - c_k is fluid (the
// forward step pulled n_k(y) from C_k(y - c_k)), and mu_{opp k}(y) goes to
// lambda_k(y) itself when y + c_k is a wall (the forward step bounced C_k(y)
// back into n_{opp k}(y)).  Every entry of lambda is written exactly once.
template <typename real>
__global__ __launch_bounds__(256) void k_adj_stream(const uint32_t* __restrict__ links, int nx,
                                                    int ny, int nz, Phys<real> ph,
                                                    const real* __restrict__ lam,
                                                    const real* __restrict__ rhof,
                                                    const real* __restrict__ qf,
                                                    const real* __restrict__ df,
                                                    const real* __restrict__ ef,
                                                    real* __restrict__ out,
                                                    double* __restrict__ partials,
                                                    int accumulate) {
  __shared__ double sh[16];
  double gab[1] = {0};
  const int N = nx * ny * nz;
  const PopGeo pg = pop_geo(nx, ny, nz);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    const uint32_t lb = links[i];
    int xs[3], ys[3], zs[3];
    axis3(i % nx, nx, xs);
    axis3((i / nx) % ny, ny, ys);
    axis3(i / (nx * ny), nz, zs);
    const uint32_t si = pop_slot(pg, zs[1], ys[1] * nx + xs[1]);
    if (lb & SELF_SOLID) {
#pragma unroll
      for (int k = 0; k < 2 * Q; ++k) out[(k / Q) * (size_t)pg.sp + si + (k % Q) * PBLK] = 0;
      continue;
    }
    real acc[2] = {0, 0};
    stencil_acc(qf, N, xs, ys, zs, nx, ny, ph, acc);
    const real e[3] = {ef[i], ef[(size_t)N + i], ef[2 * (size_t)N + i]};
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      real ps, dps;
      psi_pair(ph.psi_form, rhof[(size_t)a * N + i], ps, dps);
      const real D = df[(size_t)a * N + i] + dps * (-ph.gab * acc[a]);
      gab[0] -= (double)ps * (double)acc[a];
      const real E[3] = {ph.inv_tau[a] * e[0], ph.inv_tau[a] * e[1], ph.inv_tau[a] * e[2]};
      const real keep = real(1) - ph.inv_tau[a];
      real mu[Q];
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        // D + E . c_k, along the components c_k moves in
        const int c[3] = {CX[k], CY[k], CZ[k]};
        real m = D;
#pragma unroll
        for (int d = 0; d < 3; ++d)
          if (c[d]) m += c[d] > 0 ? E[d] : -E[d];
        mu[k] = m + keep * lam[a * (size_t)pg.sp + si + k * PBLK];
      }
      real* __restrict__ oa = out + a * (size_t)pg.sp;
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        if (!((lb >> OPP[k]) & 1u)) {  // y - c_k is fluid: it pulled n_k(y)
          const uint32_t x = pop_slot(pg, zs[1 - CZ[k]], ys[1 - CY[k]] * nx + xs[1 - CX[k]]);
          oa[x + k * PBLK] = mu[k];
        }
        if ((lb >> k) & 1u)  // y + c_k is a wall: n_{opp k}(y) came from C_k(y)
          oa[si + k * PBLK] = mu[OPP[k]];
      }
    }
  }
  block_sum_adj<1>(gab, sh);
  if (threadIdx.x == 0)
    partials[blockIdx.x * RED_STRIDE + GAB_COL] =
        accumulate ? partials[blockIdx.x * RED_STRIDE + GAB_COL] + gab[0] : gab[0];
}

// Workgroups of the local pass (grid-stride over the nodes).  The FP64
// kernel fits two waves per SIMD (its register set), so more workgroups
// than two per CU only queue; the FP32 kernel fits three.
static int adj_local_grid(size_t real_size) { return real_size == 8 ? 512 : 2048; }
// The pass that gathers the transposed stencil (and with it the g_ab
// gradient) runs one workgroup per 256 nodes up to ADJ_BLOCKS, each with its
// own row of partials.
static int adj_gather_grid(size_t N) {
  const size_t g = (N + 255) / 256;
  return (int)(g < (size_t)ADJ_BLOCKS ? g : (size_t)ADJ_BLOCKS);
}

template <typename real>
static hipError_t adjoint_t(const real* C, const real* lam_in, real* lam_out,
                            const uint32_t* links, int nx, int ny, int nz, const PhysD& phd,
                            real* rhof, real* jf, const real* mom, real* qf, real* df, real* ef,
                            double* partials, int accumulate, hipStream_t s) {
  const Phys<real> ph = phys_cast<real>(phd);
  const size_t N = (size_t)nx * ny * nz;
  const real* jm = jf;
  if (mom) {
    // moments stored by the recomputed forward step: densities, then momenta
    rhof = const_cast<real*>(mom);  // read only below
    jm = mom + 2 * N;
  } else {
    const size_t g = (N + 255) / 256;
    hipLaunchKernelGGL(k_stream_moments<real>, dim3((unsigned)(g > 8192 ? 8192 : g)), dim3(256),
                       0, s, C, links, rhof, jf, nx, ny, nz);
  }
  // FP64: the species-split local pass at two waves per SIMD (144.9 against
  // 150.7 us for one lane per node on 128 x 128 x 64); FP32 fits three waves
  // per SIMD with both species on one lane, and the split runs slower there
  // (80.1 against 50.4 us)
  if constexpr (sizeof(real) == 8)
    hipLaunchKernelGGL(k_adj_local_split<real>, dim3(adj_local_grid(sizeof(real))), dim3(256), 0, s,
                       jm, lam_in, links, rhof, nx, ny, nz, ph, qf, df, ef, partials, accumulate);
  else
    hipLaunchKernelGGL(k_adj_local<real>, dim3(adj_local_grid(sizeof(real))), dim3(256), 0, s, jm,
                       lam_in, links, rhof, nx, ny, nz, ph, qf, df, ef, partials, accumulate);
  // the transposed stencil inside the push pass (one sweep of D fewer than
  // a pass of its own), with one row of g_ab partials per workgroup
  const int blocks = adj_gather_grid(N);
  hipLaunchKernelGGL(k_adj_stream<real>, dim3(blocks), dim3(256), 0, s, links, nx, ny, nz, ph,
                     lam_in, rhof, qf, df, ef, lam_out, partials, accumulate);
  return hipGetLastError();
}

__global__ void k_sum5(const double* __restrict__ partials, int nblocks, int ngather,
                       double* __restrict__ out, double* __restrict__ acc);

hipError_t launch_adjoint(int dtype, const void* state_t, const void* lam_in, void* lam_out,
                          const uint32_t* links, int nx, int ny, int nz, const PhysD& ph,
                          void* rho_field, void* j_field, const void* mom_cached, void* q_field,
                          void* d_field, void* e_field, double* partials, double* dparams_dev,
                          double* acc_partials, hipStream_t s) {
  // with acc_partials the block partials accumulate over steps and are summed
  // only when read (launch_adjoint_sum); otherwise this step's sum goes to
  // dparams_dev
  double* part = acc_partials ? acc_partials : partials;
  const int accumulate = acc_partials != nullptr;
  hipError_t e;
  if (dtype == 0)
    e = adjoint_t<double>((const double*)state_t, (const double*)lam_in, (double*)lam_out, links,
                          nx, ny, nz, ph, (double*)rho_field, (double*)j_field,
                          (const double*)mom_cached, (double*)q_field, (double*)d_field,
                          (double*)e_field, part, accumulate, s);
  else
    e = adjoint_t<float>((const float*)state_t, (const float*)lam_in, (float*)lam_out, links, nx,
                         ny, nz, ph, (float*)rho_field, (float*)j_field, (const float*)mom_cached,
                         (float*)q_field, (float*)d_field, (float*)e_field, part, accumulate, s);
  if (e != hipSuccess) return e;
  if (accumulate) return hipSuccess;
  return launch_adjoint_sum(dtype, partials, (size_t)nx * ny * nz, dparams_dev, s);
}

hipError_t launch_adjoint_sum(int dtype, const double* partials, size_t N, double* out,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_sum5, dim3(1), dim3(256), 0, s, partials, adj_local_grid(dtype == 0 ? 8 : 4),
                     adj_gather_grid(N), out, nullptr);
  return hipGetLastError();
}

// out = this step's parameter gradient; acc (if not NULL) += out, in step order
__global__ __launch_bounds__(256) void k_sum5(const double* __restrict__ partials, int nblocks,
                                              int ngather, double* __restrict__ out,
                                              double* __restrict__ acc) {
  __shared__ double sh[5 * 16];
  double v[5] = {0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
    for (int j = 0; j < 5; ++j) v[j] += partials[b * RED_STRIDE + j];
  // the g_ab part gathered with the transposed stencil (one row per
  // workgroup of that pass)
  for (int b = threadIdx.x; b < ngather; b += blockDim.x) v[2] += partials[b * RED_STRIDE + GAB_COL];
  block_sum_adj<5>(v, sh);
  if (threadIdx.x == 0)
    for (int j = 0; j < 5; ++j) {
      out[j] = v[j];
      if (acc) acc[j] += v[j];
    }
}

__global__ void k_zero(double* __restrict__ p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0.0;
}

hipError_t launch_zero(double* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace scd
