// common.hpp -- device-side lattice tables and kernel argument structs of
// libscdrop (gfx950).  Internal header: not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scd {

// D3Q19 velocity set in the order of the public state layout: rest, the six
// axis vectors as +/- pairs, the twelve face diagonals as +/- pairs
// (Sec. 2 uses a D3Q19 lattice; weights 1/3, 1/18, 1/36 and c_s^2 = 1/3).
constexpr int Q = 19;
constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
// opposite velocity: pairs (1,2), (3,4), ..., (17,18)
constexpr int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
constexpr double WEIGHT[Q] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                              1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                              1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

// Link mask of a node (uint32): bit k (1..18) set when node x + c_k is a
// wall node, bit 0 set when x itself is a wall node.  Streaming pulls along
// c_k from x - c_k = x + c_{opp k}, so bit OPP[k] decides bounce-back.
constexpr uint32_t SELF_SOLID = 1u;

// Population buffers (the state C^a_k and the adjoint's lambda) are blocked.
// Each species holds nz planes; a plane holds ceil(nx ny / 32) blocks of 32
// consecutive plane indices c = y nx + x; a block stores its 19 velocities
// one after another, 32 values each.  Element (a, k, z, c) sits at
//   a sp + ((z pb + c / 32) 19 + k) 32 + c % 32.
// One velocity of a 32-node row is one contiguous run and the 19 velocities
// of the row share one block, so the pulls of a tile row stay within few
// DRAM pages.  The slots of the last block of a plane past nx ny are padding,
// never read.
constexpr uint32_t PBLK = 32;
struct PopGeo {
  uint32_t pb;  // blocks per plane
  uint32_t sp;  // elements per species: 19 * 32 * pb * nz
};
__host__ __device__ inline PopGeo pop_geo(int nx, int ny, int nz) {
  PopGeo g;
  g.pb = ((uint32_t)nx * (uint32_t)ny + PBLK - 1) / PBLK;
  g.sp = (uint32_t)Q * PBLK * g.pb * (uint32_t)nz;
  return g;
}
// Element offset, within one species, of velocity 0 of node (z, c); velocity
// k adds k * PBLK.
__host__ __device__ inline uint32_t pop_slot(const PopGeo& g, int z, int c) {
  return ((uint32_t)z * g.pb + ((uint32_t)c >> 5)) * (Q * PBLK) + ((uint32_t)c & (PBLK - 1));
}
// The same for a node index i = z nx ny + c (P = nx ny).
__host__ __device__ inline uint32_t pop_slot_i(const PopGeo& g, int i, int P) {
  const int z = i / P;
  return pop_slot(g, z, i - z * P);
}

// Physical parameters in the precision of the computation.
template <typename real>
struct Phys {
  real tau[2], inv_tau[2];
  real gab, gw[2];
  real psiw[2];     // psi(rho_wall^a)
  real dpsiw[2];    // psi'(rho_wall^a)
  real wa, wd;      // force weights of axis and diagonal neighbours
  int psi_form;     // 0: psi = rho, 1: psi = 1 - exp(-rho)
};

// One lattice as seen by the step kernels.
template <typename real>
struct LatDev {
  const real* __restrict__ src;   // state C^t
  real* __restrict__ dst;         // state C^{t+1}
  const uint32_t* __restrict__ links;
  int nx, ny, nz;
  int N;                          // nx * ny * nz (< 2^31)
  PopGeo geo;                     // layout of src and dst
  Phys<real> ph;
  // optional: the moments of the post-stream populations of src, as 8 fields
  // of N: rho^A, rho^B, j^A (x, y, z), j^B (x, y, z)
  real* __restrict__ mom_out;
};

template <typename real>
__device__ __forceinline__ real psi_of(int form, real rho) {
  return form == 1 ? real(1) - exp(-rho) : rho;
}
template <typename real>
__device__ __forceinline__ real dpsi_of(int form, real rho) {
  return form == 1 ? exp(-rho) : real(1);
}

__device__ __forceinline__ int wrap_index(int v, int n) {
  v = v % n;
  return v < 0 ? v + n : v;
}

// Wrapped coordinates of a node and its two neighbours along one axis:
// c[0] = v - 1, c[1] = v, c[2] = v + 1 (periodic).
__device__ __forceinline__ void axis3(int v, int n, int (&c)[3]) {
  c[1] = v;
  c[0] = v == 0 ? n - 1 : v - 1;
  c[2] = v == n - 1 ? 0 : v + 1;
}

// Node index of x + d for d in {-1, 0, 1}^3 given wrapped triples.
__device__ __forceinline__ int nbr_index(const int (&xs)[3], const int (&ys)[3], const int (&zs)[3],
                                         int nx, int ny, int dx, int dy, int dz) {
  return (zs[1 + dz] * ny + ys[1 + dy]) * nx + xs[1 + dx];
}

// Load of one value at a uniform base plus a 32-bit byte offset (lowers to
// the scalar-base + 32-bit vector-offset form of the global load).  The host
// guarantees sp * sizeof(real) < 2^32, so offsets within one species fit.
template <typename real>
__device__ __forceinline__ real ld_off(const char* __restrict__ base, uint32_t boff) {
  return *reinterpret_cast<const real*>(base + boff);
}
template <typename real>
__device__ __forceinline__ void st_off(char* __restrict__ base, uint32_t boff, real v) {
  *reinterpret_cast<real*>(base + boff) = v;
}
// Streaming store: the new state is not read again within this step, so it
// need not displace the state and halo lines the step still reads from L2.
template <typename real>
__device__ __forceinline__ void st_off_nt(char* __restrict__ base, uint32_t boff, real v) {
  __builtin_nontemporal_store(v, reinterpret_cast<real*>(base + boff));
}

// Streaming with mid-grid bounce-back (Sec. 2): the 38 post-stream
// populations of fluid node (xs[1], ys[1], zs[1]).  For each k the value
// comes from x - c_k, or from the opposite population of x itself when
// x - c_k is a wall node.
template <typename real>
__device__ __forceinline__ void pull38(const real* __restrict__ src, const PopGeo& g,
                                       const int (&xs)[3], const int (&ys)[3], const int (&zs)[3],
                                       int nx, uint32_t lb, real (&n)[38]) {
  const char* __restrict__ pa = reinterpret_cast<const char*>(src);
  const char* __restrict__ pb = reinterpret_cast<const char*>(src + g.sp);
  constexpr uint32_t S = sizeof(real);
  const uint32_t self = pop_slot(g, zs[1], ys[1] * nx + xs[1]);
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const uint32_t j = pop_slot(g, zs[1 - CZ[k]], ys[1 - CY[k]] * nx + xs[1 - CX[k]]);
    const bool bb = (lb >> OPP[k]) & 1u;
    // velocity k at node x - c_k, or velocity OPP[k] at x
    const uint32_t off = bb ? (self + (uint32_t)OPP[k] * PBLK) * S : (j + (uint32_t)k * PBLK) * S;
    n[k] = ld_off<real>(pa, off);
    n[Q + k] = ld_off<real>(pb, off);
  }
}

// Post-stream densities only (sums of the pulled populations).
template <typename real>
__device__ __forceinline__ void pull_density(const real* __restrict__ src, const PopGeo& g,
                                             const int (&xs)[3], const int (&ys)[3],
                                             const int (&zs)[3], int nx, uint32_t lb,
                                             real& ra, real& rb) {
  real n[38];
  pull38(src, g, xs, ys, zs, nx, lb, n);
  real a = 0, b = 0;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    a += n[k];
    b += n[Q + k];
  }
  ra = a;
  rb = b;
}

// Moments of one species: rho = sum_k n_k, j = sum_k n_k c_k (Sec. 2).
template <typename real>
__device__ __forceinline__ void moments(const real* n, real& rho, real& jx, real& jy, real& jz) {
  real r = 0, x = 0, y = 0, z = 0;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    r += n[k];
    if (CX[k] == 1) x += n[k];
    if (CX[k] == -1) x -= n[k];
    if (CY[k] == 1) y += n[k];
    if (CY[k] == -1) y -= n[k];
    if (CZ[k] == 1) z += n[k];
    if (CZ[k] == -1) z -= n[k];
  }
  rho = r; jx = x; jy = y; jz = z;
}

// Eq. (Equil) for the pair (k, opp k): with s = c_k.u the two equilibria
// share the even part e = 1 - 3/2 u^2 + 9/2 s^2 and differ in the sign of
// the odd part o = s (3 + 9/2 s^2 - 9/2 u^2).
template <typename real>
__device__ __forceinline__ void equilibrium_pair(real wr, real s, real uu, real& fk, real& fo) {
  real s2 = s * s;
  real e = real(1) - real(1.5) * uu + real(4.5) * s2;
  real o = s * (real(3) + real(4.5) * s2 - real(4.5) * uu);
  fk = wr * (e + o);
  fo = wr * (e - o);
}

}  // namespace scd
