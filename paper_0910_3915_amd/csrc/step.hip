// step.hip -- the fused time step of the two-component Shan-Chen D3Q19 model
// with interacting walls (Sec. 2 of the paper) on gfx950, plus the small
// kernels around it (link masks, initial equilibrium, densities).
//
// Fused step, one z-marching tile per workgroup:
//   * a workgroup owns TX x TY columns and a chunk [za, zb) of z planes;
//   * for every plane p it pulls the 38 post-stream populations of its
//     columns (streaming + mid-grid bounce-back), computes the densities and
//     the pseudopotential products e^a = G^a psi^b that the force stencil
//     needs, and writes them into a ring of 4 planes in LDS; the ring also
//     holds a one-node halo around the tile, whose densities are pulled by
//     spare threads (those reads are served by L2 since the neighbouring
//     tiles read the same lines);
//   * one barrier later plane p - 1 has e on planes p - 2, p - 1, p and is
//     collided: 18-neighbour Shan-Chen + wall force, the common velocity and
//     the velocity shift, BGK toward the third-order equilibrium, and 38
//     coalesced stores.  The pulled populations of p - 1 stay in registers.
// HBM traffic per fluid node and step is one read and one write of each
// population (plus a 4-byte link mask); everything else is on chip.
#include <cstring>

#include "common.hpp"
#include "kernels.hpp"

namespace scd {

template <typename real>
struct alignas(2 * sizeof(real)) E2 {
  real a, b;  // e^A = G^A psi^B and e^B = G^B psi^A at one node
};

template <int TX, int TY>
struct Tile {
  static constexpr int NT = TX * TY;
  static constexpr int LX = TX + 2;
  static constexpr int LY = TY + 2;
  static constexpr int P = LX * LY;          // LDS positions per plane
  static constexpr int R = 2 * LX + 2 * TY;  // halo positions per plane
  static constexpr int HPT = (R + NT - 1) / NT;
};

// e^A, e^B of a fluid node from its post-stream densities (Eq. SCforce:
// the neighbour's psi of the *other* species times the coupling).
template <typename real>
__device__ __forceinline__ E2<real> fluid_e(const Phys<real>& ph, real ra, real rb) {
  E2<real> e;
  e.a = ph.gab * psi_of(ph.psi_form, rb);
  e.b = ph.gab * psi_of(ph.psi_form, ra);
  return e;
}
// wall node: constant content, coupling g_wall^a (Sec. 2 wall model)
template <typename real>
__device__ __forceinline__ E2<real> wall_e(const Phys<real>& ph) {
  E2<real> e;
  e.a = ph.gw[0] * ph.psiw[1];
  e.b = ph.gw[1] * ph.psiw[0];
  return e;
}

// Eq. (SCforce) sums of one node from the e values of its 18 neighbours
// (read through the three plane pointers of the LDS ring):
// S^a = sum_k W_k e^a(x + c_k) c_k.
template <typename real, int LX>
__device__ __forceinline__ void force_sums(const Phys<real>& ph, const E2<real>* __restrict__ sm,
                                           const E2<real>* __restrict__ s0,
                                           const E2<real>* __restrict__ sp, int pos,
                                           real (&S)[6]) {
  real sax = 0, say = 0, saz = 0, sbx = 0, sby = 0, sbz = 0;
#pragma unroll
  for (int k = 1; k < Q; ++k) {
    const E2<real>* s = CZ[k] < 0 ? sm : (CZ[k] > 0 ? sp : s0);
    E2<real> e = s[pos + CY[k] * LX + CX[k]];
    real w = (CX[k] * CX[k] + CY[k] * CY[k] + CZ[k] * CZ[k]) == 1 ? ph.wa : ph.wd;
    real wa = w * e.a, wb = w * e.b;
    if (CX[k]) { sax += CX[k] * wa; sbx += CX[k] * wb; }
    if (CY[k]) { say += CY[k] * wa; sby += CY[k] * wb; }
    if (CZ[k]) { saz += CZ[k] * wa; sbz += CZ[k] * wb; }
  }
  S[0] = sax; S[1] = say; S[2] = saz; S[3] = sbx; S[4] = sby; S[5] = sbz;
}

// Keeps the compiler from moving instructions across this point, so that
// the phases of a node update do not all hold their registers at once.
__device__ __forceinline__ void phase_fence() { __builtin_amdgcn_sched_barrier(0); }

// Collision of one fluid node given its post-stream populations n and the
// force sums S of Eq. (SCforce).
template <typename real>
__device__ __forceinline__ void collide_node(const LatDev<real>& L, const real (&n)[38],
                                             const real (&Sf)[6], int i) {
  const Phys<real>& ph = L.ph;
  real ra, jax, jay, jaz, rb, jbx, jby, jbz;
  moments(&n[0], ra, jax, jay, jaz);
  moments(&n[Q], rb, jbx, jby, jbz);
  const real sax = Sf[0], say = Sf[1], saz = Sf[2], sbx = Sf[3], sby = Sf[4], sbz = Sf[5];
  const real pa = psi_of(ph.psi_form, ra), pb = psi_of(ph.psi_form, rb);
  const real fax = -pa * sax, fay = -pa * say, faz = -pa * saz;
  const real fbx = -pb * sbx, fby = -pb * sby, fbz = -pb * sbz;
  // common velocity u' = sum_a j^a / tau^a / sum_a rho^a / tau^a, then the
  // velocity shift u^a = u' + tau^a F^a / rho^a (Sec. 2)
  const real itA = ph.inv_tau[0], itB = ph.inv_tau[1];
  const real iR = real(1) / (ra * itA + rb * itB);
  const real upx = (jax * itA + jbx * itB) * iR;
  const real upy = (jay * itA + jby * itB) * iR;
  const real upz = (jaz * itA + jbz * itB) * iR;
  const real sA = ph.tau[0] / ra, sB = ph.tau[1] / rb;
  real u[2][3] = {{upx + sA * fax, upy + sA * fay, upz + sA * faz},
                  {upx + sB * fbx, upy + sB * fby, upz + sB * fbz}};
  const real rho[2] = {ra, rb};
  constexpr uint32_t S = sizeof(real);
  const uint32_t si = pop_slot_i(L.geo, i, L.nx * L.ny);
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const real ux = u[a][0], uy = u[a][1], uz = u[a][2];
    const real uu = ux * ux + uy * uy + uz * uz;
    const real it = ph.inv_tau[a];
    char* __restrict__ out = reinterpret_cast<char*>(L.dst + (size_t)a * L.geo.sp);
    real moving = 0;  // sum of the 18 moving equilibria
#pragma unroll
    for (int k = 1; k < Q; k += 2) {
      const int o = k + 1;  // OPP[k] for odd k
      real s = CX[k] * ux + CY[k] * uy + CZ[k] * uz;
      real fk, fo;
      equilibrium_pair(real(WEIGHT[k]) * rho[a], s, uu, fk, fo);
      moving += fk + fo;
      real nk = n[a * Q + k], no = n[a * Q + o];
      st_off<real>(out, (si + (uint32_t)k * PBLK) * S, nk + (fk - nk) * it);
      st_off<real>(out, (si + (uint32_t)o * PBLK) * S, no + (fo - no) * it);
    }
    // rest population: the equilibrium's zeroth moment is rho exactly, so
    // n^eq_0 = rho - sum of the moving ones (the same value as
    // zeta_0 rho (1 - 3/2 u^2) in exact arithmetic, and mass-exact in
    // floating point where the weights 1/3, 1/18, 1/36 are not)
    const real eq0 = rho[a] - moving;
    const real f0 = n[a * Q];
    st_off<real>(out, si * S, f0 + (eq0 - f0) * it);
  }
}

// Variants of the z-march:
//   REG    -- the pulled populations of the plane being collided stay in
//             registers while the next plane is pulled (two sets live);
//   REPULL -- the look-ahead plane is pulled for its densities only and the
//             collided plane is pulled again (from L2 / the last-level
//             cache): one set live, so more waves fit on a SIMD.
constexpr int VAR_REG = 0;
[[maybe_unused]] constexpr int VAR_REPULL = 1;

// One z-marching tile of the fused step (shared by the single-lattice and
// the batched kernels).  lds: 4 * Tile::P entries.
template <typename real, int TX, int TY, int VAR>
__device__ __forceinline__ void step_tile(const LatDev<real>& L, int bx, int by, int za, int zb,
                                          E2<real>* __restrict__ lds) {
  using T = Tile<TX, TY>;
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  const int x0 = bx * TX, y0 = by * TY;
  const bool active = (x0 + tx) < nx && (y0 + ty) < ny;
  // lanes past the first column or row beyond a partial tile's edge feed
  // no active node: they act as wall nodes (no pulls, never collided)
  const bool need = (x0 + tx) <= nx && (y0 + ty) <= ny;
  int xs[3], ys[3];
  axis3(wrap_index(x0 + tx, nx), nx, xs);
  axis3(wrap_index(y0 + ty, ny), ny, ys);
  const int pos = (ty + 1) * T::LX + (tx + 1);

  // halo positions served by this thread
  int hx[T::HPT][3], hy[T::HPT][3], hpos[T::HPT];
  bool hval[T::HPT];
  // halo positions are dealt wave-major: consecutive lanes take consecutive
  // halo nodes, the first waves take all of them and the others issue no
  // halo loads (no wave pulls more than HPT nodes either way)
#pragma unroll
  for (int h = 0; h < T::HPT; ++h) {
    const int q = tid + h * T::NT;
    const bool valid = q < T::R;
    int lx, ly;
    if (q < T::LX) { ly = -1; lx = q - 1; }
    else if (q < 2 * T::LX) { ly = TY; lx = q - T::LX - 1; }
    else if (q < 2 * T::LX + TY) { lx = -1; ly = q - 2 * T::LX; }
    else { lx = TX; ly = q - 2 * T::LX - TY; }
    // a halo node no active node of the tile reads (past the first column
    // or row beyond a partial tile's edge) is left out: no loads, no e
    hval[h] = valid && x0 + lx <= nx && y0 + ly <= ny;
    if (!hval[h]) { lx = 0; ly = 0; }
    axis3(wrap_index(x0 + lx, nx), nx, hx[h]);
    axis3(wrap_index(y0 + ly, ny), ny, hy[h]);
    hpos[h] = (ly + 1) * T::LX + (lx + 1);
  }

  const E2<real> ewall = wall_e(L.ph);
  real ncur[38], nnext[38];
  bool solid_cur = true, solid_next = true;

  // Link masks of the plane about to be pulled, loaded one plane ahead so
  // that the population loads of a plane never wait for its masks.
  uint32_t lbi, lbh[T::HPT];
  auto load_links = [&](int zr, uint32_t& li, uint32_t(&lh)[T::HPT]) {
    const int z = wrap_index(zr, nz);
    li = need ? L.links[(z * ny + ys[1]) * nx + xs[1]] : SELF_SOLID;
#pragma unroll
    for (int h = 0; h < T::HPT; ++h)
      lh[h] = hval[h] ? L.links[(z * ny + hy[h][1]) * nx + hx[h][1]] : SELF_SOLID;
  };
  load_links(za - 1, lbi, lbh);

  // e of plane zr (raw, may lie outside [0, nz)) into ring slot zr & 3; the
  // interior populations are kept in nout when keep is set.  All loads of
  // the plane (halo and interior) are issued before any of them is used,
  // then the masks of plane zr + 1 are requested.
  auto plane = [&](int zr, bool keep, real(&nout)[38], bool& solid_out) {
    int zs[3];
    axis3(wrap_index(zr, nz), nz, zs);
    E2<real>* slot = lds + (zr & 3) * T::P;
    real hm[T::HPT][38];
#pragma unroll
    for (int h = 0; h < T::HPT; ++h)
      if (!(lbh[h] & SELF_SOLID)) pull38(L.src, L.geo, hx[h], hy[h], zs, nx, lbh[h], hm[h]);
    solid_out = (lbi & SELF_SOLID) != 0;
    real m[38];
    if (!solid_out) {
      if (keep) pull38(L.src, L.geo, xs, ys, zs, nx, lbi, nout);
      else pull38(L.src, L.geo, xs, ys, zs, nx, lbi, m);
    }
    uint32_t nli, nlh[T::HPT];
    load_links(zr + 1, nli, nlh);
#pragma unroll
    for (int h = 0; h < T::HPT; ++h) {
      if (!hval[h]) continue;
      E2<real> e = ewall;
      if (!(lbh[h] & SELF_SOLID)) {
        real ra = 0, rb = 0;
#pragma unroll
        for (int k = 0; k < Q; ++k) { ra += hm[h][k]; rb += hm[h][Q + k]; }
        e = fluid_e(L.ph, ra, rb);
      }
      slot[hpos[h]] = e;
    }
    E2<real> e = ewall;
    if (!solid_out) {
      real ra = 0, rb = 0;
      if (keep) {
#pragma unroll
        for (int k = 0; k < Q; ++k) { ra += nout[k]; rb += nout[Q + k]; }
      } else {
#pragma unroll
        for (int k = 0; k < Q; ++k) { ra += m[k]; rb += m[Q + k]; }
      }
      e = fluid_e(L.ph, ra, rb);
    }
    slot[pos] = e;
    lbi = nli;
#pragma unroll
    for (int h = 0; h < T::HPT; ++h) lbh[h] = nlh[h];
  };

  if constexpr (VAR == VAR_REG) {
    plane(za - 1, false, nnext, solid_next);
    plane(za, true, ncur, solid_cur);
    for (int p = za + 1; p <= zb; ++p) {
      plane(p, p < zb, nnext, solid_next);
      __syncthreads();
      const int zc = p - 1;
      if (active && !solid_cur) {
        const int i = (zc * ny + ys[1]) * nx + xs[1];
        real S[6];
        force_sums<real, T::LX>(L.ph, lds + ((zc - 1) & 3) * T::P, lds + (zc & 3) * T::P,
                                lds + ((zc + 1) & 3) * T::P, pos, S);
        collide_node<real>(L, ncur, S, i);
      }
#pragma unroll
      for (int k = 0; k < 38; ++k) ncur[k] = nnext[k];
      solid_cur = solid_next;
    }
  } else {
    plane(za - 1, false, nnext, solid_next);
    plane(za, false, nnext, solid_next);
    for (int p = za + 1; p <= zb; ++p) {
      plane(p, false, nnext, solid_next);
      __syncthreads();
      const int zc = p - 1;
      if (active) {
        int zs[3];
        axis3(zc, nz, zs);
        const int i = (zc * ny + ys[1]) * nx + xs[1];
        const uint32_t lb = L.links[i];
        if (!(lb & SELF_SOLID)) {
          real S[6];
          force_sums<real, T::LX>(L.ph, lds + ((zc - 1) & 3) * T::P, lds + (zc & 3) * T::P,
                                  lds + ((zc + 1) & 3) * T::P, pos, S);
          phase_fence();
          pull38(L.src, L.geo, xs, ys, zs, nx, lb, ncur);
          collide_node<real>(L, ncur, S, i);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Species-split z-march.  Each wave covers 32 nodes of a tile row: lanes
// 0-31 carry species A, lanes 32-63 species B of the same nodes, so every
// thread pulls, collides and stores the 19 populations of one species, and
// one load instruction reads two contiguous 32-node segments.  The two
// species of a node meet through a cross-half-wave swap (__shfl_xor by 32)
// of their density and momentum.  A thread of species a writes e^{b} =
// G^{b} psi^{a} of its node into the LDS ring (the value the *other*
// species' force needs), so halo nodes need no exchange at all: a halo task
// pulls one species' 19 populations of one node.
template <typename real>
__device__ __forceinline__ void pull19(const real* __restrict__ src, const PopGeo& g, int a,
                                       const int (&xs)[3], const int (&ys)[3], const int (&zs)[3],
                                       int nx, uint32_t lb, real (&n)[19]) {
  const char* __restrict__ base = reinterpret_cast<const char*>(src + (size_t)a * g.sp);
  constexpr uint32_t S = sizeof(real);
  const uint32_t self = pop_slot(g, zs[1], ys[1] * nx + xs[1]);
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const uint32_t j = pop_slot(g, zs[1 - CZ[k]], ys[1 - CY[k]] * nx + xs[1 - CX[k]]);
    const bool bb = (lb >> OPP[k]) & 1u;
    const uint32_t off = bb ? (self + (uint32_t)OPP[k] * PBLK) * S : (j + (uint32_t)k * PBLK) * S;
    n[k] = ld_off<real>(base, off);
  }
}

// e value written by a thread of species a: what species b = 1 - a feels
// from this node (Eq. SCforce at fluid nodes, the wall model at walls).
template <typename real>
__device__ __forceinline__ real e_from(const Phys<real>& ph, int a, bool wall, real rho_a) {
  const int b = 1 - a;
  return wall ? ph.gw[b] * ph.psiw[a] : ph.gab * psi_of(ph.psi_form, rho_a);
}

template <int TX, int TY>
struct SplitTile {
  static constexpr int NODES = TX * TY;
  static constexpr int NT = 2 * NODES;  // threads
  static constexpr int LX = TX + 2;
  static constexpr int P = LX * (TY + 2);
  static constexpr int R = 2 * LX + 2 * TY;           // halo nodes
  static constexpr int TASKS = 2 * R;                  // halo (node, species) pulls
  static constexpr int HPT = (TASKS + NT - 1) / NT;
  static_assert(TX % 32 == 0, "a half-wave covers 32 nodes of one row");
};

template <typename real, int TX, int TY, bool NT_STORE, bool JOINT>
__device__ __forceinline__ void step_tile_split(const LatDev<real>& L, int bx, int by, int za,
                                                int zb, real* __restrict__ lds, int dir = 1) {
  auto store = [](char* base, uint32_t off, real v) {
    if constexpr (NT_STORE) st_off_nt<real>(base, off, v);
    else st_off<real>(base, off, v);
  };
  using T = SplitTile<TX, TY>;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int a = lane >> 5;                          // species of this thread
  const int node = wave * 32 + (lane & 31);         // node of the tile
  const int tx = node % TX, ty = node / TX;
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  const int x0 = bx * TX, y0 = by * TY;
  const bool active = (x0 + tx) < nx && (y0 + ty) < ny;
  // lanes past the first column or row beyond a partial tile's edge feed
  // no active node: they act as wall nodes (no pulls, never collided)
  const bool need = (x0 + tx) <= nx && (y0 + ty) <= ny;
  int xs[3], ys[3];
  axis3(wrap_index(x0 + tx, nx), nx, xs);
  axis3(wrap_index(y0 + ty, ny), ny, ys);
  const int pos = (ty + 1) * T::LX + (tx + 1);
  // LDS ring: 4 planes x 2 species x P positions; plane slot s, species c
  auto ring = [&](int zr, int c) { return lds + ((zr & 3) * 2 + c) * T::P; };

  // halo tasks dealt wave-major as the interior: lanes 0-31 of a wave take
  // species 0 of 32 consecutive halo nodes, lanes 32-63 species 1
  int hx[T::HPT][3], hy[T::HPT][3], hpos[T::HPT], hsp[T::HPT];
  bool hval[T::HPT];
#pragma unroll
  for (int h = 0; h < T::HPT; ++h) {
    const int sl = tid + h * T::NT;
    const int q = (sl >> 6) * 32 + (sl & 31);
    const bool valid = q < T::R;
    hsp[h] = (sl >> 5) & 1;
    int lx, ly;
    if (q < T::LX) { ly = -1; lx = q - 1; }
    else if (q < 2 * T::LX) { ly = TY; lx = q - T::LX - 1; }
    else if (q < 2 * T::LX + TY) { lx = -1; ly = q - 2 * T::LX; }
    else { lx = TX; ly = q - 2 * T::LX - TY; }
    // a halo node no active node of the tile reads (past the first column
    // or row beyond a partial tile's edge) is left out: no loads, no e
    hval[h] = valid && x0 + lx <= nx && y0 + ly <= ny;
    if (!hval[h]) { lx = 0; ly = 0; }
    axis3(wrap_index(x0 + lx, nx), nx, hx[h]);
    axis3(wrap_index(y0 + ly, ny), ny, hy[h]);
    hpos[h] = (ly + 1) * T::LX + (lx + 1);
  }

  real ncur[19], nnext[19];
  bool solid_cur = true, solid_next = true;

  // Link masks of the plane about to be pulled, loaded one plane ahead so
  // that the population loads of a plane never wait for its masks.
  uint32_t lbi, lbh[T::HPT];
  auto load_links = [&](int zr, uint32_t& li, uint32_t(&lh)[T::HPT]) {
    const int z = wrap_index(zr, nz);
    li = need ? L.links[(z * ny + ys[1]) * nx + xs[1]] : SELF_SOLID;
#pragma unroll
    for (int h = 0; h < T::HPT; ++h)
      lh[h] = hval[h] ? L.links[(z * ny + hy[h][1]) * nx + hx[h][1]] : SELF_SOLID;
  };
  load_links(dir > 0 ? za - 1 : zb, lbi, lbh);

  // Parameters of the e values, held in registers for the whole march.
  const real gab = L.ph.gab;
  const int psi_form = L.ph.psi_form;
  const real ew0 = L.ph.gw[1] * L.ph.psiw[0];  // e written by a wall thread of species 0
  const real ew1 = L.ph.gw[0] * L.ph.psiw[1];  // ... of species 1
  auto e_of = [&](int sp, bool wall, real rho) {
    return wall ? (sp ? ew1 : ew0) : gab * psi_of(psi_form, rho);
  };

  // The halo of plane zr is pulled and reduced first, then the interior
  // (a fence between them bounds the live registers: the interior set is
  // pulled while the collided plane's set is still held); the masks of the
  // next plane of the march are requested behind the interior loads.
  auto plane_fenced = [&](int zr, bool keep, real(&nout)[19], bool& solid_out) {
    int zs[3];
    axis3(wrap_index(zr, nz), nz, zs);
#pragma unroll
    for (int h = 0; h < T::HPT; ++h) {
      if (!hval[h]) continue;
      const bool wall = lbh[h] & SELF_SOLID;
      real r = 0;
      if (!wall) {
        real m[19];
        pull19(L.src, L.geo, hsp[h], hx[h], hy[h], zs, nx, lbh[h], m);
#pragma unroll
        for (int k = 0; k < Q; ++k) r += m[k];
      }
      ring(zr, 1 - hsp[h])[hpos[h]] = e_from(L.ph, hsp[h], wall, r);
    }
    phase_fence();
    solid_out = (lbi & SELF_SOLID) != 0;
    real m[19];
    if (!solid_out) {
      if (keep) pull19(L.src, L.geo, a, xs, ys, zs, nx, lbi, nout);
      else pull19(L.src, L.geo, a, xs, ys, zs, nx, lbi, m);
    }
    load_links(zr + dir, lbi, lbh);
    real r = 0;
    if (!solid_out) {
      if (keep) {
#pragma unroll
        for (int k = 0; k < Q; ++k) r += nout[k];
      } else {
#pragma unroll
        for (int k = 0; k < Q; ++k) r += m[k];
      }
    }
    ring(zr, 1 - a)[pos] = e_from(L.ph, a, solid_out, r);
  };

  // All loads of plane zr are issued before any is used: the interior set,
  // then the halo, then the masks of the next plane of the march.
  auto plane_joint = [&](int zr, bool keep, real(&nout)[19], bool& solid_out) {
    int zs[3];
    axis3(wrap_index(zr, nz), nz, zs);
    solid_out = (lbi & SELF_SOLID) != 0;
    real m[19];
    if (!solid_out) {
      if (keep) pull19(L.src, L.geo, a, xs, ys, zs, nx, lbi, nout);
      else pull19(L.src, L.geo, a, xs, ys, zs, nx, lbi, m);
    }
    real hm[T::HPT][19];
#pragma unroll
    for (int h = 0; h < T::HPT; ++h) {
      if (!(lbh[h] & SELF_SOLID))
        pull19(L.src, L.geo, hsp[h], hx[h], hy[h], zs, nx, lbh[h], hm[h]);
    }
    uint32_t nli, nlh[T::HPT];
    load_links(zr + dir, nli, nlh);
    real r = 0;
    if (!solid_out) {
      if (keep) {
#pragma unroll
        for (int k = 0; k < Q; ++k) r += nout[k];
      } else {
#pragma unroll
        for (int k = 0; k < Q; ++k) r += m[k];
      }
    }
    ring(zr, 1 - a)[pos] = e_of(a, solid_out, r);
#pragma unroll
    for (int h = 0; h < T::HPT; ++h) {
      if (!hval[h]) continue;
      const bool wall = lbh[h] & SELF_SOLID;
      real rh = 0;
      if (!wall) {
#pragma unroll
        for (int k = 0; k < Q; ++k) rh += hm[h][k];
      }
      ring(zr, 1 - hsp[h])[hpos[h]] = e_of(hsp[h], wall, rh);
    }
    lbi = nli;
#pragma unroll
    for (int h = 0; h < T::HPT; ++h) lbh[h] = nlh[h];
  };

  auto plane = [&](int zr, bool keep, real(&nout)[19], bool& solid_out) {
    if constexpr (JOINT) plane_joint(zr, keep, nout, solid_out);
    else plane_fenced(zr, keep, nout, solid_out);
  };

  // March up (dir = 1) from za - 1 or down (dir = -1) from zb; the planes
  // of [za, zb) are collided, each once all three of its e planes are in.
  const Phys<real>& ph = L.ph;
  const int first = dir > 0 ? za - 1 : zb, last = dir > 0 ? zb : za - 1;
  plane(first, false, nnext, solid_next);
  plane(first + dir, true, ncur, solid_cur);
  for (int p = first + 2 * dir; dir > 0 ? p <= last : p >= last; p += dir) {
    plane(p, dir > 0 ? p < zb : p >= za, nnext, solid_next);
    __syncthreads();
    const int zc = p - dir;
    // every lane takes part in the swap; inactive and wall lanes carry zeros
    real rho, jx, jy, jz;
    moments(ncur, rho, jx, jy, jz);
    const real rho_o = __shfl_xor(rho, 32, 64), jx_o = __shfl_xor(jx, 32, 64);
    const real jy_o = __shfl_xor(jy, 32, 64), jz_o = __shfl_xor(jz, 32, 64);
    if (active && !solid_cur) {
      // Eq. (SCforce) on species a: S^a = sum_k W_k e^a(x + c_k) c_k
      const real* sm = ring(zc - 1, a);
      const real* s0 = ring(zc, a);
      const real* sp = ring(zc + 1, a);
      real sx = 0, sy = 0, sz = 0;
#pragma unroll
      for (int k = 1; k < Q; ++k) {
        const real* s = CZ[k] < 0 ? sm : (CZ[k] > 0 ? sp : s0);
        const real w = (CX[k] * CX[k] + CY[k] * CY[k] + CZ[k] * CZ[k]) == 1 ? ph.wa : ph.wd;
        const real e = w * s[pos + CY[k] * T::LX + CX[k]];
        if (CX[k]) sx += CX[k] * e;
        if (CY[k]) sy += CY[k] * e;
        if (CZ[k]) sz += CZ[k] * e;
      }
      const real psi_a = psi_of(ph.psi_form, rho);
      // the common velocity, with the two species in a fixed order so that
      // both halves of the wave compute the same value
      const real rA = a ? rho_o : rho, rB = a ? rho : rho_o;
      const real jAx = a ? jx_o : jx, jBx = a ? jx : jx_o;
      const real jAy = a ? jy_o : jy, jBy = a ? jy : jy_o;
      const real jAz = a ? jz_o : jz, jBz = a ? jz : jz_o;
      const real itA = ph.inv_tau[0], itB = ph.inv_tau[1];
      const real iR = real(1) / (rA * itA + rB * itB);
      const real sh = ph.tau[a] / rho;
      const real ux = (jAx * itA + jBx * itB) * iR + sh * (-psi_a * sx);
      const real uy = (jAy * itA + jBy * itB) * iR + sh * (-psi_a * sy);
      const real uz = (jAz * itA + jBz * itB) * iR + sh * (-psi_a * sz);
      const real uu = ux * ux + uy * uy + uz * uz;
      const real it = ph.inv_tau[a];
      const uint32_t si = pop_slot(L.geo, zc, ys[1] * nx + xs[1]);
      char* __restrict__ out = reinterpret_cast<char*>(L.dst + (size_t)a * L.geo.sp);
      constexpr uint32_t S = sizeof(real);
      real moving = 0;
#pragma unroll
      for (int k = 1; k < Q; k += 2) {
        const int o = k + 1;
        const real s = CX[k] * ux + CY[k] * uy + CZ[k] * uz;
        real fk, fo;
        equilibrium_pair(real(WEIGHT[k]) * rho, s, uu, fk, fo);
        moving += fk + fo;
        store(out, (si + (uint32_t)k * PBLK) * S, ncur[k] + (fk - ncur[k]) * it);
        store(out, (si + (uint32_t)o * PBLK) * S, ncur[o] + (fo - ncur[o]) * it);
      }
      const real eq0 = rho - moving;
      store(out, si * S, ncur[0] + (eq0 - ncur[0]) * it);
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) ncur[k] = nnext[k];
    solid_cur = solid_next;
  }
}

// ---------------------------------------------------------------------------
// Species-split z-march G planes at a time: each iteration issues the loads
// of the next G planes (interior and halo) together, then collides G planes
// after one barrier, so a wave keeps G times the bytes in flight per memory
// latency and meets one barrier per G planes.  The e ring has RS plane slots
// (RS >= 2G + 2): an iteration writes the slots of its G new planes while
// the previous iteration's collisions may still read the G + 2 before them.
// Byte offsets of the nine columns (x + dx, y + dy) around a node within one
// z plane of one species, indexed [1 + dy][1 + dx]: with a plane's byte
// offset, every neighbour of the node is one addition away.
template <typename real>
__device__ __forceinline__ void column_offsets(const PopGeo& g, const int (&xs)[3],
                                               const int (&ys)[3], int nx, uint32_t (&o)[3][3]) {
#pragma unroll
  for (int dy = 0; dy < 3; ++dy)
#pragma unroll
    for (int dx = 0; dx < 3; ++dx)
      o[dy][dx] = pop_slot(g, 0, ys[dy] * nx + xs[dx]) * (uint32_t)sizeof(real);
}

// The pull of pull19 from precomputed column offsets and the byte offsets
// zo of planes z - 1, z, z + 1: the neighbour and the bounce-back offsets
// are each one addition, so the choice between them is a select.
template <typename real>
__device__ __forceinline__ void pull19_cols(const char* __restrict__ base, uint32_t NS,
                                            const uint32_t (&col)[3][3], const uint32_t (&zo)[3],
                                            uint32_t lb, real (&n)[19]) {
  const uint32_t self = zo[1] + col[1][1];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const uint32_t nb = (uint32_t)k * NS + zo[1 - CZ[k]] + col[1 - CY[k]][1 - CX[k]];
    const uint32_t bb = (uint32_t)OPP[k] * NS + self;
    n[k] = ld_off<real>(base, ((lb >> OPP[k]) & 1u) ? bb : nb);
  }
}

template <int G>
struct MultiRing {
  static constexpr int RS = G <= 3 ? 8 : 16;
  static_assert(RS >= 2 * G + 2, "ring too short for the planes in flight");
};

template <typename real, int TX, int TY, int G>
__device__ __forceinline__ void step_tile_multi(const LatDev<real>& L, int bx, int by, int za,
                                                int zb, real* __restrict__ lds, int dir = 1) {
  using T = SplitTile<TX, TY>;
  constexpr int RS = MultiRing<G>::RS;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int a = lane >> 5;
  const int node = wave * 32 + (lane & 31);
  const int tx = node % TX, ty = node / TX;
  const int nx = L.nx, ny = L.ny, nz = L.nz, N = L.N;
  const int x0 = bx * TX, y0 = by * TY;
  const bool active = (x0 + tx) < nx && (y0 + ty) < ny;
  // lanes past the first column or row beyond a partial tile's edge feed
  // no active node: they act as wall nodes (no pulls, never collided)
  const bool need = (x0 + tx) <= nx && (y0 + ty) <= ny;
  int xs[3], ys[3];
  axis3(wrap_index(x0 + tx, nx), nx, xs);
  axis3(wrap_index(y0 + ty, ny), ny, ys);
  const int pos = (ty + 1) * T::LX + (tx + 1);
  auto ring = [&](int zr, int c) { return lds + ((zr & (RS - 1)) * 2 + c) * T::P; };

  // Halo tasks are dealt wave-major, laid out like the interior: lanes 0-31
  // of a wave take species 0 of 32 consecutive halo nodes, lanes 32-63
  // species 1 of the same nodes.  The first waves take all of them, so the
  // others issue no halo loads, and each half-wave reads one run of nodes.
  int hx[T::HPT][3], hy[T::HPT][3], hpos[T::HPT], hsp[T::HPT];
  bool hval[T::HPT];
#pragma unroll
  for (int h = 0; h < T::HPT; ++h) {
    const int sl = tid + h * T::NT;
    const int q = (sl >> 6) * 32 + (sl & 31);
    const bool valid = q < T::R;
    hsp[h] = (sl >> 5) & 1;
    int lx, ly;
    if (q < T::LX) { ly = -1; lx = q - 1; }
    else if (q < 2 * T::LX) { ly = TY; lx = q - T::LX - 1; }
    else if (q < 2 * T::LX + TY) { lx = -1; ly = q - 2 * T::LX; }
    else { lx = TX; ly = q - 2 * T::LX - TY; }
    // a halo node no active node of the tile reads (past the first column
    // or row beyond a partial tile's edge) is left out: no loads, no e
    hval[h] = valid && x0 + lx <= nx && y0 + ly <= ny;
    if (!hval[h]) { lx = 0; ly = 0; }
    axis3(wrap_index(x0 + lx, nx), nx, hx[h]);
    axis3(wrap_index(y0 + ly, ny), ny, hy[h]);
    hpos[h] = (ly + 1) * T::LX + (lx + 1);
  }

  // byte offsets: one velocity (NS), one z plane (PS), the columns around the
  // thread's node and halo nodes; per-species bases of the source state
  constexpr uint32_t S = sizeof(real);
  const uint32_t NS = PBLK * S, PS = L.geo.pb * (Q * PBLK) * S;
  uint32_t col[3][3], hcol[T::HPT][3][3];
  column_offsets<real>(L.geo, xs, ys, nx, col);
  const char* __restrict__ sbase = reinterpret_cast<const char*>(L.src + (size_t)a * L.geo.sp);
  const char* __restrict__ hbase[T::HPT];
  int hidx[T::HPT];
#pragma unroll
  for (int h = 0; h < T::HPT; ++h) {
    column_offsets<real>(L.geo, hx[h], hy[h], nx, hcol[h]);
    hbase[h] = reinterpret_cast<const char*>(L.src + (size_t)hsp[h] * L.geo.sp);
    hidx[h] = hy[h][1] * nx + hx[h][1];
  }
  const int cidx = ys[1] * nx + xs[1];

  // the march: plane j = 0 .. M + 1 in march order, interior planes 1 .. M
  const int M = zb - za;
  auto zof = [&](int j) { return dir > 0 ? za - 1 + j : zb - j; };
  auto links_of = [&](int j, uint32_t& li, uint32_t(&lh)[T::HPT]) {
    const int zn = wrap_index(zof(j), nz) * nx * ny;
    li = need ? L.links[zn + cidx] : SELF_SOLID;
#pragma unroll
    for (int h = 0; h < T::HPT; ++h) lh[h] = hval[h] ? L.links[zn + hidx[h]] : SELF_SOLID;
  };

  const real gab = L.ph.gab;
  const int psi_form = L.ph.psi_form;
  const real ew0 = L.ph.gw[1] * L.ph.psiw[0];  // e written by a wall thread of species 0
  const real ew1 = L.ph.gw[0] * L.ph.psiw[1];  // ... of species 1
  auto e_of = [&](int sp, bool wall, real rho) {
    return wall ? (sp ? ew1 : ew0) : gab * psi_of(psi_form, rho);
  };

  // loads of plane j into n (interior) and hm (halo)
  auto issue = [&](int j, uint32_t li, const uint32_t(&lh)[T::HPT], real(&n)[19],
                   real(&hm)[T::HPT][19]) {
    int zs[3];
    axis3(wrap_index(zof(j), nz), nz, zs);
    const uint32_t zo[3] = {(uint32_t)zs[0] * PS, (uint32_t)zs[1] * PS, (uint32_t)zs[2] * PS};
    if (!(li & SELF_SOLID)) pull19_cols<real>(sbase, NS, col, zo, li, n);
#pragma unroll
    for (int h = 0; h < T::HPT; ++h)
      if (!(lh[h] & SELF_SOLID)) pull19_cols<real>(hbase[h], NS, hcol[h], zo, lh[h], hm[h]);
  };
  // densities of plane j -> e values into its ring slot (and, when asked
  // for, the densities of the chunk's own planes to mom_out)
  auto reduce = [&](int j, uint32_t li, const uint32_t(&lh)[T::HPT], const real(&n)[19],
                    const real(&hm)[T::HPT][19]) {
    const int zr = zof(j);
    const bool wall = li & SELF_SOLID;
    real r = 0;
    if (!wall) {
#pragma unroll
      for (int k = 0; k < Q; ++k) r += n[k];
    }
    ring(zr, 1 - a)[pos] = e_of(a, wall, r);
    if (L.mom_out && j >= 1 && j <= M && active)
      L.mom_out[(size_t)a * N + (size_t)zr * nx * ny + cidx] = r;
#pragma unroll
    for (int h = 0; h < T::HPT; ++h) {
      if (!hval[h]) continue;
      const bool hw = lh[h] & SELF_SOLID;
      real rh = 0;
      if (!hw) {
#pragma unroll
        for (int k = 0; k < Q; ++k) rh += hm[h][k];
      }
      ring(zr, 1 - hsp[h])[hpos[h]] = e_of(hsp[h], hw, rh);
    }
  };

  const Phys<real>& ph = L.ph;
  auto collide = [&](int zc, const real(&nc)[19], bool solid) {
    // every lane takes part in the swap; inactive and wall lanes carry junk
    real rho, jx, jy, jz;
    moments(nc, rho, jx, jy, jz);
    const real rho_o = __shfl_xor(rho, 32, 64), jx_o = __shfl_xor(jx, 32, 64);
    const real jy_o = __shfl_xor(jy, 32, 64), jz_o = __shfl_xor(jz, 32, 64);
    if (!active || solid) return;
    if (L.mom_out) {
      real* m = L.mom_out + (size_t)(2 + 3 * a) * N + (size_t)zc * nx * ny + cidx;
      m[0] = jx;
      m[N] = jy;
      m[2 * (size_t)N] = jz;
    }
    // Eq. (SCforce) on species a: S^a = sum_k W_k e^a(x + c_k) c_k
    const real* sm = ring(zc - 1, a);
    const real* s0 = ring(zc, a);
    const real* sp = ring(zc + 1, a);
    real sx = 0, sy = 0, sz = 0;
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      const real* sl = CZ[k] < 0 ? sm : (CZ[k] > 0 ? sp : s0);
      const real w = (CX[k] * CX[k] + CY[k] * CY[k] + CZ[k] * CZ[k]) == 1 ? ph.wa : ph.wd;
      const real e = w * sl[pos + CY[k] * T::LX + CX[k]];
      if (CX[k]) sx += CX[k] * e;
      if (CY[k]) sy += CY[k] * e;
      if (CZ[k]) sz += CZ[k] * e;
    }
    const real psi_a = psi_of(ph.psi_form, rho);
    // the common velocity, with the two species in a fixed order so that
    // both halves of the wave compute the same value
    const real rA = a ? rho_o : rho, rB = a ? rho : rho_o;
    const real jAx = a ? jx_o : jx, jBx = a ? jx : jx_o;
    const real jAy = a ? jy_o : jy, jBy = a ? jy : jy_o;
    const real jAz = a ? jz_o : jz, jBz = a ? jz : jz_o;
    const real itA = ph.inv_tau[0], itB = ph.inv_tau[1];
    const real iR = real(1) / (rA * itA + rB * itB);
    const real shf = ph.tau[a] / rho;
    const real ux = (jAx * itA + jBx * itB) * iR + shf * (-psi_a * sx);
    const real uy = (jAy * itA + jBy * itB) * iR + shf * (-psi_a * sy);
    const real uz = (jAz * itA + jBz * itB) * iR + shf * (-psi_a * sz);
    const real uu = ux * ux + uy * uy + uz * uz;
    const real it = ph.inv_tau[a];
    const uint32_t iS = (uint32_t)zc * PS + col[1][1];
    char* __restrict__ out = reinterpret_cast<char*>(L.dst + (size_t)a * L.geo.sp);
    real moving = 0;
#pragma unroll
    for (int k = 1; k < Q; k += 2) {
      const int o = k + 1;
      const real sdot = CX[k] * ux + CY[k] * uy + CZ[k] * uz;
      real fk, fo;
      equilibrium_pair(real(WEIGHT[k]) * rho, sdot, uu, fk, fo);
      moving += fk + fo;
      st_off_nt<real>(out, (uint32_t)k * NS + iS, nc[k] + (fk - nc[k]) * it);
      st_off_nt<real>(out, (uint32_t)o * NS + iS, nc[o] + (fo - nc[o]) * it);
    }
    const real eq0 = rho - moving;
    st_off_nt<real>(out, iS, nc[0] + (eq0 - nc[0]) * it);
  };

  // n[0]: the plane collided first in an iteration; n[g]: plane c + g
  real n[G + 1][19];
  real hm[G][T::HPT][19];
  bool solid[G + 1];
  uint32_t lk[G], lkh[G][T::HPT];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    lk[g] = SELF_SOLID;
#pragma unroll
    for (int h = 0; h < T::HPT; ++h) lkh[g][h] = SELF_SOLID;
  }
  // prologue: planes 0 and 1 (plane 0 only feeds e values), masks of 2 .. G + 1
  {
    uint32_t l0, lh0[T::HPT], l1, lh1[T::HPT];
    links_of(0, l0, lh0);
    links_of(1, l1, lh1);
    issue(0, l0, lh0, n[1], hm[0]);
    issue(1, l1, lh1, n[0], hm[G - 1]);
    reduce(0, l0, lh0, n[1], hm[0]);
    reduce(1, l1, lh1, n[0], hm[G - 1]);
    solid[0] = (l1 & SELF_SOLID) != 0;
  }
#pragma unroll
  for (int g = 0; g < G; ++g)
    if (2 + g <= M + 1) links_of(2 + g, lk[g], lkh[g]);
  // iteration: pull planes c + 1 .. c + G, collide planes c .. c + G - 1
  for (int c = 1; c <= M; c += G) {
    uint32_t u[G], uh[G][T::HPT];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      u[g] = lk[g];
#pragma unroll
      for (int h = 0; h < T::HPT; ++h) uh[g][h] = lkh[g][h];
    }
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (c + 1 + g <= M + 1) issue(c + 1 + g, u[g], uh[g], n[1 + g], hm[g]);
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (c + 1 + G + g <= M + 1) links_of(c + 1 + G + g, lk[g], lkh[g]);
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (c + 1 + g <= M + 1) {
        reduce(c + 1 + g, u[g], uh[g], n[1 + g], hm[g]);
        solid[1 + g] = (u[g] & SELF_SOLID) != 0;
      }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (c + g <= M) collide(zof(c + g), n[g], solid[g]);
    // plane c + G opens the next iteration
#pragma unroll
    for (int k = 0; k < Q; ++k) n[0][k] = n[G][k];
    solid[0] = solid[G];
  }
}

// ---------------------------------------------------------------------------
// The species-split multi-plane march on a tile of TY rows in which each
// thread owns RR nodes of one column, TY / RR rows apart.  A TX x TY tile
// then runs on the threads of a TX x (TY / RR) one, so that a taller tile,
// with fewer halo nodes per interior node, fits the registers of one wave
// per SIMD: a 32 x 8 tile has 84 halo nodes for 256 interior ones (0.33
// per node) against 76 for 128 (0.59) on 32 x 4.  Per iteration the loads
// of G planes of all RR rows are in flight together, as in the G-plane march.
template <typename real, int TX, int TY, int G, int RR>
__device__ __forceinline__ void step_tile_rows(const LatDev<real>& L, int bx, int by, int za,
                                               int zb, real* __restrict__ lds, int dir = 1) {
  using T = SplitTile<TX, TY>;  // geometry of the whole tile (ring, halo)
  constexpr int TYT = TY / RR;  // thread rows
  static_assert(TY % RR == 0, "rows per thread must divide the tile height");
  constexpr int NT = 2 * TX * TYT;
  constexpr int HPT = (T::TASKS + NT - 1) / NT;
  constexpr int RS = MultiRing<G>::RS;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int a = lane >> 5;
  const int node = wave * 32 + (lane & 31);
  const int tx = node % TX, ty0 = node / TX;
  const int nx = L.nx, ny = L.ny, nz = L.nz, N = L.N;
  const int x0 = bx * TX, y0 = by * TY;
  bool active[RR], need[RR];
  int xs[3], ys[RR][3], pos[RR];
  axis3(wrap_index(x0 + tx, nx), nx, xs);
#pragma unroll
  for (int r = 0; r < RR; ++r) {
    const int ty = ty0 + r * TYT;
    active[r] = (x0 + tx) < nx && (y0 + ty) < ny;
    // lanes past the first column or row beyond a partial tile's edge feed
    // no active node: they act as wall nodes (no pulls, never collided)
    need[r] = (x0 + tx) <= nx && (y0 + ty) <= ny;
    axis3(wrap_index(y0 + ty, ny), ny, ys[r]);
    pos[r] = (ty + 1) * T::LX + (tx + 1);
  }
  auto ring = [&](int zr, int c) { return lds + ((zr & (RS - 1)) * 2 + c) * T::P; };

  // halo tasks dealt wave-major over the NT threads, as in the G-plane march
  int hx[HPT][3], hy[HPT][3], hpos[HPT], hsp[HPT];
  bool hval[HPT];
#pragma unroll
  for (int h = 0; h < HPT; ++h) {
    const int sl = tid + h * NT;
    const int q = (sl >> 6) * 32 + (sl & 31);
    const bool valid = q < T::R;
    hsp[h] = (sl >> 5) & 1;
    int lx, ly;
    if (q < T::LX) { ly = -1; lx = q - 1; }
    else if (q < 2 * T::LX) { ly = TY; lx = q - T::LX - 1; }
    else if (q < 2 * T::LX + TY) { lx = -1; ly = q - 2 * T::LX; }
    else { lx = TX; ly = q - 2 * T::LX - TY; }
    hval[h] = valid && x0 + lx <= nx && y0 + ly <= ny;
    if (!hval[h]) { lx = 0; ly = 0; }
    axis3(wrap_index(x0 + lx, nx), nx, hx[h]);
    axis3(wrap_index(y0 + ly, ny), ny, hy[h]);
    hpos[h] = (ly + 1) * T::LX + (lx + 1);
  }

  constexpr uint32_t S = sizeof(real);
  const uint32_t NS = PBLK * S, PS = L.geo.pb * (Q * PBLK) * S;
  uint32_t col[RR][3][3], hcol[HPT][3][3];
  int cidx[RR];
#pragma unroll
  for (int r = 0; r < RR; ++r) {
    column_offsets<real>(L.geo, xs, ys[r], nx, col[r]);
    cidx[r] = ys[r][1] * nx + xs[1];
  }
  const char* __restrict__ sbase = reinterpret_cast<const char*>(L.src + (size_t)a * L.geo.sp);
  const char* __restrict__ hbase[HPT];
  int hidx[HPT];
#pragma unroll
  for (int h = 0; h < HPT; ++h) {
    column_offsets<real>(L.geo, hx[h], hy[h], nx, hcol[h]);
    hbase[h] = reinterpret_cast<const char*>(L.src + (size_t)hsp[h] * L.geo.sp);
    hidx[h] = hy[h][1] * nx + hx[h][1];
  }

  const int M = zb - za;
  auto zof = [&](int j) { return dir > 0 ? za - 1 + j : zb - j; };
  auto links_of = [&](int j, uint32_t(&li)[RR], uint32_t(&lh)[HPT]) {
    const int zn = wrap_index(zof(j), nz) * nx * ny;
#pragma unroll
    for (int r = 0; r < RR; ++r) li[r] = need[r] ? L.links[zn + cidx[r]] : SELF_SOLID;
#pragma unroll
    for (int h = 0; h < HPT; ++h) lh[h] = hval[h] ? L.links[zn + hidx[h]] : SELF_SOLID;
  };

  const real gab = L.ph.gab;
  const int psi_form = L.ph.psi_form;
  const real ew0 = L.ph.gw[1] * L.ph.psiw[0];
  const real ew1 = L.ph.gw[0] * L.ph.psiw[1];
  auto e_of = [&](int sp, bool wall, real rho) {
    return wall ? (sp ? ew1 : ew0) : gab * psi_of(psi_form, rho);
  };

  auto issue = [&](int j, const uint32_t(&li)[RR], const uint32_t(&lh)[HPT], real(&n)[RR][19],
                   real(&hm)[HPT][19]) {
    int zs[3];
    axis3(wrap_index(zof(j), nz), nz, zs);
    const uint32_t zo[3] = {(uint32_t)zs[0] * PS, (uint32_t)zs[1] * PS, (uint32_t)zs[2] * PS};
#pragma unroll
    for (int r = 0; r < RR; ++r)
      if (!(li[r] & SELF_SOLID)) pull19_cols<real>(sbase, NS, col[r], zo, li[r], n[r]);
#pragma unroll
    for (int h = 0; h < HPT; ++h)
      if (!(lh[h] & SELF_SOLID)) pull19_cols<real>(hbase[h], NS, hcol[h], zo, lh[h], hm[h]);
  };
  auto reduce = [&](int j, const uint32_t(&li)[RR], const uint32_t(&lh)[HPT], const real(&n)[RR][19],
                    const real(&hm)[HPT][19]) {
    const int zr = zof(j);
#pragma unroll
    for (int r = 0; r < RR; ++r) {
      const bool wall = li[r] & SELF_SOLID;
      real rho = 0;
      if (!wall) {
#pragma unroll
        for (int k = 0; k < Q; ++k) rho += n[r][k];
      }
      ring(zr, 1 - a)[pos[r]] = e_of(a, wall, rho);
      if (L.mom_out && j >= 1 && j <= M && active[r])
        L.mom_out[(size_t)a * N + (size_t)zr * nx * ny + cidx[r]] = rho;
    }
#pragma unroll
    for (int h = 0; h < HPT; ++h) {
      if (!hval[h]) continue;
      const bool hw = lh[h] & SELF_SOLID;
      real rh = 0;
      if (!hw) {
#pragma unroll
        for (int k = 0; k < Q; ++k) rh += hm[h][k];
      }
      ring(zr, 1 - hsp[h])[hpos[h]] = e_of(hsp[h], hw, rh);
    }
  };

  const Phys<real>& ph = L.ph;
  auto collide = [&](int zc, int r, const real(&nc)[19], bool solid) {
    real rho, jx, jy, jz;
    moments(nc, rho, jx, jy, jz);
    const real rho_o = __shfl_xor(rho, 32, 64), jx_o = __shfl_xor(jx, 32, 64);
    const real jy_o = __shfl_xor(jy, 32, 64), jz_o = __shfl_xor(jz, 32, 64);
    if (!active[r] || solid) return;
    const int cx = cidx[r];
    if (L.mom_out) {
      real* m = L.mom_out + (size_t)(2 + 3 * a) * N + (size_t)zc * nx * ny + cx;
      m[0] = jx;
      m[N] = jy;
      m[2 * (size_t)N] = jz;
    }
    const real* sm = ring(zc - 1, a);
    const real* s0 = ring(zc, a);
    const real* sp = ring(zc + 1, a);
    const int ps = pos[r];
    real sx = 0, sy = 0, sz = 0;
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      const real* sl = CZ[k] < 0 ? sm : (CZ[k] > 0 ? sp : s0);
      const real w = (CX[k] * CX[k] + CY[k] * CY[k] + CZ[k] * CZ[k]) == 1 ? ph.wa : ph.wd;
      const real e = w * sl[ps + CY[k] * T::LX + CX[k]];
      if (CX[k]) sx += CX[k] * e;
      if (CY[k]) sy += CY[k] * e;
      if (CZ[k]) sz += CZ[k] * e;
    }
    const real psi_a = psi_of(ph.psi_form, rho);
    const real rA = a ? rho_o : rho, rB = a ? rho : rho_o;
    const real jAx = a ? jx_o : jx, jBx = a ? jx : jx_o;
    const real jAy = a ? jy_o : jy, jBy = a ? jy : jy_o;
    const real jAz = a ? jz_o : jz, jBz = a ? jz : jz_o;
    const real itA = ph.inv_tau[0], itB = ph.inv_tau[1];
    const real iR = real(1) / (rA * itA + rB * itB);
    const real shf = ph.tau[a] / rho;
    const real ux = (jAx * itA + jBx * itB) * iR + shf * (-psi_a * sx);
    const real uy = (jAy * itA + jBy * itB) * iR + shf * (-psi_a * sy);
    const real uz = (jAz * itA + jBz * itB) * iR + shf * (-psi_a * sz);
    const real uu = ux * ux + uy * uy + uz * uz;
    const real it = ph.inv_tau[a];
    const uint32_t iS = (uint32_t)zc * PS + col[r][1][1];
    char* __restrict__ out = reinterpret_cast<char*>(L.dst + (size_t)a * L.geo.sp);
    real moving = 0;
#pragma unroll
    for (int k = 1; k < Q; k += 2) {
      const int o = k + 1;
      const real sdot = CX[k] * ux + CY[k] * uy + CZ[k] * uz;
      real fk, fo;
      equilibrium_pair(real(WEIGHT[k]) * rho, sdot, uu, fk, fo);
      moving += fk + fo;
      st_off_nt<real>(out, (uint32_t)k * NS + iS, nc[k] + (fk - nc[k]) * it);
      st_off_nt<real>(out, (uint32_t)o * NS + iS, nc[o] + (fo - nc[o]) * it);
    }
    const real eq0 = rho - moving;
    st_off_nt<real>(out, iS, nc[0] + (eq0 - nc[0]) * it);
  };

  // n[g][r]: plane c + g of row r (n[0]: the plane collided first)
  real n[G + 1][RR][19];
  real hm[G][HPT][19];
  bool solid[G + 1][RR];
  uint32_t lk[G][RR], lkh[G][HPT];
#pragma unroll
  for (int g = 0; g < G; ++g) {
#pragma unroll
    for (int r = 0; r < RR; ++r) lk[g][r] = SELF_SOLID;
#pragma unroll
    for (int h = 0; h < HPT; ++h) lkh[g][h] = SELF_SOLID;
  }
  {
    uint32_t l0[RR], lh0[HPT], l1[RR], lh1[HPT];
    links_of(0, l0, lh0);
    links_of(1, l1, lh1);
    // plane 0 only feeds e values; its halo buffer is reduced before plane
    // 1 reuses it (with G = 1 there is one)
    issue(0, l0, lh0, n[1], hm[0]);
    reduce(0, l0, lh0, n[1], hm[0]);
    issue(1, l1, lh1, n[0], hm[G - 1]);
    reduce(1, l1, lh1, n[0], hm[G - 1]);
#pragma unroll
    for (int r = 0; r < RR; ++r) solid[0][r] = (l1[r] & SELF_SOLID) != 0;
  }
#pragma unroll
  for (int g = 0; g < G; ++g)
    if (2 + g <= M + 1) links_of(2 + g, lk[g], lkh[g]);
  for (int c = 1; c <= M; c += G) {
    uint32_t u[G][RR], uh[G][HPT];
#pragma unroll
    for (int g = 0; g < G; ++g) {
#pragma unroll
      for (int r = 0; r < RR; ++r) u[g][r] = lk[g][r];
#pragma unroll
      for (int h = 0; h < HPT; ++h) uh[g][h] = lkh[g][h];
    }
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (c + 1 + g <= M + 1) issue(c + 1 + g, u[g], uh[g], n[1 + g], hm[g]);
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (c + 1 + G + g <= M + 1) links_of(c + 1 + G + g, lk[g], lkh[g]);
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (c + 1 + g <= M + 1) {
        reduce(c + 1 + g, u[g], uh[g], n[1 + g], hm[g]);
#pragma unroll
        for (int r = 0; r < RR; ++r) solid[1 + g][r] = (u[g][r] & SELF_SOLID) != 0;
      }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (c + g <= M) {
#pragma unroll
        for (int r = 0; r < RR; ++r) collide(zof(c + g), r, n[g][r], solid[g][r]);
      }
#pragma unroll
    for (int r = 0; r < RR; ++r) {
#pragma unroll
      for (int k = 0; k < Q; ++k) n[0][r][k] = n[G][r][k];
      solid[0][r] = solid[G][r];
    }
  }
}

// ---------------------------------------------------------------------------
// Software-pipelined species-split z-march.  Iteration p issues the loads of
// plane p (interior and halo), collides plane p - 2 while they are in
// flight, then turns plane p into e values.  Collision of plane c needs e
// on planes c - 1, c, c + 1, all written before the barrier that ended
// iteration c + 1; iteration p writes ring slot p & 3 while the collision
// reads slots (p - 3, p - 2, p - 1) & 3, so one barrier per plane suffices.
// Three population sets are live per thread (planes p - 2, p - 1, p).
template <typename real, int TX, int TY>
__device__ __forceinline__ void step_tile_pipe(const LatDev<real>& L, int bx, int by, int za,
                                               int zb, real* __restrict__ lds) {
  using T = SplitTile<TX, TY>;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int a = lane >> 5;
  const int node = wave * 32 + (lane & 31);
  const int tx = node % TX, ty = node / TX;
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  const int x0 = bx * TX, y0 = by * TY;
  const bool active = (x0 + tx) < nx && (y0 + ty) < ny;
  // lanes past the first column or row beyond a partial tile's edge feed
  // no active node: they act as wall nodes (no pulls, never collided)
  const bool need = (x0 + tx) <= nx && (y0 + ty) <= ny;
  int xs[3], ys[3];
  axis3(wrap_index(x0 + tx, nx), nx, xs);
  axis3(wrap_index(y0 + ty, ny), ny, ys);
  const int pos = (ty + 1) * T::LX + (tx + 1);
  auto ring = [&](int zr, int c) { return lds + ((zr & 3) * 2 + c) * T::P; };

  // halo tasks dealt wave-major as in the species-split march
  int hx[T::HPT][3], hy[T::HPT][3], hpos[T::HPT], hsp[T::HPT];
  bool hval[T::HPT];
#pragma unroll
  for (int h = 0; h < T::HPT; ++h) {
    const int sl = tid + h * T::NT;
    const int q = (sl >> 6) * 32 + (sl & 31);
    const bool valid = q < T::R;
    hsp[h] = (sl >> 5) & 1;
    int lx, ly;
    if (q < T::LX) { ly = -1; lx = q - 1; }
    else if (q < 2 * T::LX) { ly = TY; lx = q - T::LX - 1; }
    else if (q < 2 * T::LX + TY) { lx = -1; ly = q - 2 * T::LX; }
    else { lx = TX; ly = q - 2 * T::LX - TY; }
    // a halo node no active node of the tile reads (past the first column
    // or row beyond a partial tile's edge) is left out: no loads, no e
    hval[h] = valid && x0 + lx <= nx && y0 + ly <= ny;
    if (!hval[h]) { lx = 0; ly = 0; }
    axis3(wrap_index(x0 + lx, nx), nx, hx[h]);
    axis3(wrap_index(y0 + ly, ny), ny, hy[h]);
    hpos[h] = (ly + 1) * T::LX + (lx + 1);
  }
  const Phys<real>& ph = L.ph;

  real n0[19], n1[19], n2[19];       // planes p - 2, p - 1, p
  real hm[T::HPT][19];               // halo pulls of plane p
  bool s0 = true, s1 = true, s2 = true;
  bool hw[T::HPT];

  // issue the loads of plane zr (halo and interior)
  auto load_plane = [&](int zr, real(&nout)[19], bool& solid_out) {
    int zs[3];
    axis3(wrap_index(zr, nz), nz, zs);
#pragma unroll
    for (int h = 0; h < T::HPT; ++h) {
      hw[h] = true;
      if (!hval[h]) continue;
      const int i = (zs[1] * ny + hy[h][1]) * nx + hx[h][1];
      const uint32_t lb = L.links[i];
      hw[h] = lb & SELF_SOLID;
      if (!hw[h]) pull19(L.src, L.geo, hsp[h], hx[h], hy[h], zs, nx, lb, hm[h]);
    }
    const int i = (zs[1] * ny + ys[1]) * nx + xs[1];
    const uint32_t lb = need ? L.links[i] : SELF_SOLID;
    solid_out = (lb & SELF_SOLID) != 0;
    if (!solid_out) pull19(L.src, L.geo, a, xs, ys, zs, nx, lb, nout);
  };
  // e values of plane zr from the loaded populations
  auto finish_plane = [&](int zr, const real(&nin)[19], bool solid_in) {
#pragma unroll
    for (int h = 0; h < T::HPT; ++h) {
      if (!hval[h]) continue;
      real r = 0;
      if (!hw[h]) {
#pragma unroll
        for (int k = 0; k < Q; ++k) r += hm[h][k];
      }
      ring(zr, 1 - hsp[h])[hpos[h]] = e_from(ph, hsp[h], hw[h], r);
    }
    real r = 0;
    if (!solid_in) {
#pragma unroll
      for (int k = 0; k < Q; ++k) r += nin[k];
    }
    ring(zr, 1 - a)[pos] = e_from(ph, a, solid_in, r);
  };
  auto collide = [&](int zc, const real(&n)[19], bool solid) {
    real rho, jx, jy, jz;
    moments(n, rho, jx, jy, jz);
    const real rho_o = __shfl_xor(rho, 32, 64), jx_o = __shfl_xor(jx, 32, 64);
    const real jy_o = __shfl_xor(jy, 32, 64), jz_o = __shfl_xor(jz, 32, 64);
    if (!active || solid) return;
    const real* sm = ring(zc - 1, a);
    const real* sc = ring(zc, a);
    const real* sp = ring(zc + 1, a);
    real sx = 0, sy = 0, sz = 0;
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      const real* s = CZ[k] < 0 ? sm : (CZ[k] > 0 ? sp : sc);
      const real w = (CX[k] * CX[k] + CY[k] * CY[k] + CZ[k] * CZ[k]) == 1 ? ph.wa : ph.wd;
      const real e = w * s[pos + CY[k] * T::LX + CX[k]];
      if (CX[k]) sx += CX[k] * e;
      if (CY[k]) sy += CY[k] * e;
      if (CZ[k]) sz += CZ[k] * e;
    }
    const real psi_a = psi_of(ph.psi_form, rho);
    const real rA = a ? rho_o : rho, rB = a ? rho : rho_o;
    const real jAx = a ? jx_o : jx, jBx = a ? jx : jx_o;
    const real jAy = a ? jy_o : jy, jBy = a ? jy : jy_o;
    const real jAz = a ? jz_o : jz, jBz = a ? jz : jz_o;
    const real itA = ph.inv_tau[0], itB = ph.inv_tau[1];
    const real iR = real(1) / (rA * itA + rB * itB);
    const real shf = ph.tau[a] / rho;
    const real ux = (jAx * itA + jBx * itB) * iR + shf * (-psi_a * sx);
    const real uy = (jAy * itA + jBy * itB) * iR + shf * (-psi_a * sy);
    const real uz = (jAz * itA + jBz * itB) * iR + shf * (-psi_a * sz);
    const real uu = ux * ux + uy * uy + uz * uz;
    const real it = ph.inv_tau[a];
    const uint32_t si = pop_slot(L.geo, zc, ys[1] * nx + xs[1]);
    char* __restrict__ out = reinterpret_cast<char*>(L.dst + (size_t)a * L.geo.sp);
    constexpr uint32_t S = sizeof(real);
    real moving = 0;
#pragma unroll
    for (int k = 1; k < Q; k += 2) {
      const int o = k + 1;
      const real s = CX[k] * ux + CY[k] * uy + CZ[k] * uz;
      real fk, fo;
      equilibrium_pair(real(WEIGHT[k]) * rho, s, uu, fk, fo);
      moving += fk + fo;
      st_off_nt<real>(out, (si + (uint32_t)k * PBLK) * S, n[k] + (fk - n[k]) * it);
      st_off_nt<real>(out, (si + (uint32_t)o * PBLK) * S, n[o] + (fo - n[o]) * it);
    }
    const real eq0 = rho - moving;
    st_off_nt<real>(out, si * S, n[0] + (eq0 - n[0]) * it);
  };

  // prologue: planes za - 1 and za
  load_plane(za - 1, n1, s1);
  finish_plane(za - 1, n1, s1);
  load_plane(za, n1, s1);
  finish_plane(za, n1, s1);
  __syncthreads();
  for (int p = za + 1; p <= zb + 1; ++p) {
    const bool have = p <= zb;  // plane p is still needed for its e values
    if (have) load_plane(p, n2, s2);
    phase_fence();
    if (p - 2 >= za) collide(p - 2, n0, s0);
    phase_fence();
    if (have) finish_plane(p, n2, s2);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < Q; ++k) { n0[k] = n1[k]; n1[k] = n2[k]; }
    s0 = s1;
    s1 = s2;
  }
}

// Map the hardware block id to a tile.  Workgroups are handed to the 8 XCDs
// round-robin; with remap each XCD receives one contiguous range of tiles
// (z-chunk fastest, then x, then y), so the chunks of a column, which share
// their boundary planes, and neighbouring columns, which share halo lines,
// sit in one XCD's L2.
__device__ __forceinline__ bool tile_of_block(int b, int total, int remap, int gx, int gz, int& bx,
                                              int& by, int& bz) {
  if (remap) {
    int per = (total + 7) / 8;
    b = (b & 7) * per + (b >> 3);
    if (b >= total) return false;
  }
  bz = b % gz;
  bx = (b / gz) % gx;
  by = b / (gz * gx);
  return true;
}

constexpr int VAR_SPLIT = 2;     // species-split z-march
constexpr int VAR_SPLIT_NT = 3;  // the same with streaming stores
constexpr int VAR_PIPE = 4;      // software-pipelined species split, streaming stores
constexpr int VAR_JOINT = 5;     // species split, streaming stores, all loads of a plane
                                 // (interior and halo) issued before any is used
constexpr int VAR_DUAL = 6;      // species split, two planes per iteration
constexpr int VAR_TRIPLE = 7;    // species split, three planes per iteration
constexpr int VAR_QUAD = 8;      // species split, four planes per iteration
constexpr int VAR_ROWS2 = 9;     // two planes per iteration, two rows per thread
constexpr int VAR_ROWS1 = 10;    // one plane per iteration, two rows per thread
constexpr int VAR_ROWS4 = 11;    // one plane per iteration, four rows per thread

template <typename real, int TX, int TY, int VAR>
struct StepShape {
  static constexpr int RR = VAR == VAR_ROWS4 ? 4 : (VAR == VAR_ROWS2 || VAR == VAR_ROWS1) ? 2 : 1;
  static constexpr bool ROWS = RR > 1;  // several rows per thread
  static constexpr bool SPLIT =
      VAR == VAR_SPLIT || VAR == VAR_SPLIT_NT || VAR == VAR_PIPE || VAR == VAR_JOINT ||
      VAR == VAR_DUAL || VAR == VAR_TRIPLE || VAR == VAR_QUAD || ROWS;
  static constexpr int THREADS = ROWS ? 2 * TX * TY / RR : SPLIT ? 2 * TX * TY : TX * TY;
  static constexpr int LDS_REALS =
      VAR == VAR_DUAL || VAR == VAR_ROWS2 ? 2 * MultiRing<2>::RS * SplitTile<TX, TY>::P
      : VAR == VAR_TRIPLE                 ? 2 * MultiRing<3>::RS * SplitTile<TX, TY>::P
      : VAR == VAR_QUAD                   ? 2 * MultiRing<4>::RS * SplitTile<TX, TY>::P
      : VAR == VAR_ROWS1 || VAR == VAR_ROWS4 ? 2 * MultiRing<1>::RS * SplitTile<TX, TY>::P
      : SPLIT                             ? 8 * SplitTile<TX, TY>::P
                                          : 8 * Tile<TX, TY>::P;
};

template <typename real, int TX, int TY, int VAR>
__device__ __forceinline__ void run_tile(const LatDev<real>& L, int bx, int by, int za, int zb,
                                         real* lds, int dir = 1) {
  if constexpr (VAR == VAR_SPLIT)
    step_tile_split<real, TX, TY, false, false>(L, bx, by, za, zb, lds, dir);
  else if constexpr (VAR == VAR_SPLIT_NT)
    step_tile_split<real, TX, TY, true, false>(L, bx, by, za, zb, lds, dir);
  else if constexpr (VAR == VAR_JOINT)
    step_tile_split<real, TX, TY, true, true>(L, bx, by, za, zb, lds, dir);
  else if constexpr (VAR == VAR_DUAL)
    step_tile_multi<real, TX, TY, 2>(L, bx, by, za, zb, lds, dir);
  else if constexpr (VAR == VAR_TRIPLE)
    step_tile_multi<real, TX, TY, 3>(L, bx, by, za, zb, lds, dir);
  else if constexpr (VAR == VAR_QUAD)
    step_tile_multi<real, TX, TY, 4>(L, bx, by, za, zb, lds, dir);
  else if constexpr (VAR == VAR_ROWS2)
    step_tile_rows<real, TX, TY, 2, 2>(L, bx, by, za, zb, lds, dir);
  else if constexpr (VAR == VAR_ROWS1)
    step_tile_rows<real, TX, TY, 1, 2>(L, bx, by, za, zb, lds, dir);
  else if constexpr (VAR == VAR_ROWS4)
    step_tile_rows<real, TX, TY, 1, 4>(L, bx, by, za, zb, lds, dir);
  else if constexpr (VAR == VAR_PIPE)
    step_tile_pipe<real, TX, TY>(L, bx, by, za, zb, lds);
  else
    step_tile<real, TX, TY, VAR>(L, bx, by, za, zb, reinterpret_cast<E2<real>*>(lds));
}

template <typename real, int TX, int TY, int VAR, int WPE>
__global__ __launch_bounds__((StepShape<real, TX, TY, VAR>::THREADS))
__attribute__((amdgpu_waves_per_eu(WPE, 8)))
void k_step(LatDev<real> L, int gx, int gy, int nchunks, int zc, int remap) {
  __shared__ __align__(16) real lds[StepShape<real, TX, TY, VAR>::LDS_REALS];
  int bx, by, bz;
  if (!tile_of_block(blockIdx.x, gx * gy * nchunks, remap, gx, nchunks, bx, by, bz)) return;
  const int za = bz * zc;
  const int zb = min(za + zc, L.nz);
  // even chunks march down, odd ones up: two neighbouring chunks (adjacent
  // workgroups, one XCD) reach their shared boundary planes at the same time
  // -- both at the start or both at the end -- so one pull of those planes
  // from HBM serves both through L2
  run_tile<real, TX, TY, VAR>(L, bx, by, za, zb, lds, (bz & 1) || nchunks == 1 ? 1 : -1);
}

// Batched: the grid walks the (member, tile) items of up to BATCH_DESC_MAX
// lattices, one item per workgroup at a time (a persistent grid when it is
// shorter than the list).  Member m owns items start[m] .. start[m + 1] - 1,
// its gx * gy tile columns cut into gz chunks of zc planes, in the order of
// the single-lattice step (chunks of a column adjacent, then x, then y), and
// even chunks march down, odd ones up, as there.  The descriptors and this
// table travel by value in the kernel arguments, like the single-lattice
// step's: read from the argument segment, the descriptors' pointers are
// known to address global memory (so the tile's loads and stores take the
// global scalar-base + vector-offset forms; read from a table in device
// memory they would be flat accesses), and a workgroup finds its tile with
// no memory access before its first pull.  With remap, slot s of the walk
// takes item (s mod 8) * per + s / 8, so that each XCD (blocks are dealt to
// the 8 XCDs round-robin, and a persistent grid is a multiple of 8) works
// through one contiguous range of the list.
template <typename real>
struct BatchDescs {
  LatDev<real> L[BATCH_DESC_MAX];
  int start[BATCH_DESC_MAX + 1];
  int gx[BATCH_DESC_MAX], gz[BATCH_DESC_MAX], zc[BATCH_DESC_MAX];
  int n;
};
static_assert(sizeof(BatchDescs<double>) <= 4000, "descriptors exceed the kernel argument space");

template <typename real, int TX, int TY, int VAR, int WPE>
__global__ __launch_bounds__((StepShape<real, TX, TY, VAR>::THREADS))
__attribute__((amdgpu_waves_per_eu(WPE, 8)))
void k_step_batch(const BatchDescs<real> D, int remap) {
  __shared__ __align__(16) real lds[StepShape<real, TX, TY, VAR>::LDS_REALS];
  const int nitems = D.start[D.n];
  const int per = (nitems + 7) / 8;
  const int slots = remap ? 8 * per : nitems;
  for (int s = blockIdx.x; s < slots; s += gridDim.x) {
    const int it = remap ? (s & 7) * per + (s >> 3) : s;
    if (it >= nitems) continue;
    int m = 0;
    while (m + 1 < D.n && it >= D.start[m + 1]) ++m;
    const LatDev<real>& L = D.L[m];
    const int local = it - D.start[m], gz = D.gz[m], gx = D.gx[m];
    const int bz = local % gz, bx = (local / gz) % gx, by = local / (gz * gx);
    const int za = bz * D.zc[m];
    const int zb = min(za + D.zc[m], L.nz);
    run_tile<real, TX, TY, VAR>(L, bx, by, za, zb, lds, (bz & 1) || gz == 1 ? 1 : -1);
    __syncthreads();  // the next item rewrites the LDS ring
  }
}

// ----------------------------------------------------------------------------
__global__ void k_links(const uint8_t* __restrict__ solid, uint32_t* __restrict__ links, int nx,
                        int ny, int nz) {
  const int N = nx * ny * nz;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    const int x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
    int xs[3], ys[3], zs[3];
    axis3(x, nx, xs);
    axis3(y, ny, ys);
    axis3(z, nz, zs);
    uint32_t lb = solid[i] ? SELF_SOLID : 0u;
#pragma unroll
    for (int k = 1; k < Q; ++k)
      if (solid[nbr_index(xs, ys, zs, nx, ny, CX[k], CY[k], CZ[k])]) lb |= 1u << k;
    links[i] = lb;
  }
}

// Sec. 2 initial state: fluid at rest, C_k = zeta_k rho.
template <typename real>
__global__ void k_init(real* __restrict__ pop, const double* __restrict__ ra,
                       const double* __restrict__ rb, const uint32_t* __restrict__ links, int N,
                       int P, PopGeo g) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    const bool solid = links[i] & SELF_SOLID;
    const size_t si = pop_slot_i(g, i, P);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      pop[si + k * PBLK] = solid ? real(0) : real(WEIGHT[k] * ra[i]);
      pop[g.sp + si + k * PBLK] = solid ? real(0) : real(WEIGHT[k] * rb[i]);
    }
  }
}

// Between the blocked population layout and the plain one, element
// (a * 19 + k) * N + i.  Threads run over the plain index, node fastest, so
// both sides are read and written in runs of 32 or more.  Padding slots of
// the blocked buffer are left as they are.
template <typename real, bool TO_BLOCKED>
__global__ void k_pop_repack(const real* __restrict__ src, real* __restrict__ dst, int N, int P,
                             PopGeo g) {
  const size_t total = (size_t)2 * Q * N;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int q = (int)(e / N), i = (int)(e - (size_t)q * N);
    const size_t b = (q / Q) * (size_t)g.sp + pop_slot_i(g, i, P) + (q % Q) * PBLK;
    if (TO_BLOCKED) dst[b] = src[e];
    else dst[e] = src[b];
  }
}

// rho^a = sum_k C_k^a of the stored state, FP64 output rho[a * N + i].
template <typename real>
__global__ void k_density(const real* __restrict__ pop, const uint32_t* __restrict__ links,
                          double* __restrict__ rho, int N, int P, PopGeo g) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    double ra = 0, rb = 0;
    if (!(links[i] & SELF_SOLID)) {
      const size_t si = pop_slot_i(g, i, P);
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        ra += (double)pop[si + k * PBLK];
        rb += (double)pop[g.sp + si + k * PBLK];
      }
    }
    rho[i] = ra;
    rho[(size_t)N + i] = rb;
  }
}

// Post-stream densities of every fluid node (0 at wall nodes), rho[a*N + i].
template <typename real>
__global__ void k_stream_density(const real* __restrict__ pop, const uint32_t* __restrict__ links,
                                 real* __restrict__ rho, int nx, int ny, int nz) {
  const int N = nx * ny * nz;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    const uint32_t lb = links[i];
    real ra = 0, rb = 0;
    if (!(lb & SELF_SOLID)) {
      int xs[3], ys[3], zs[3];
      axis3(i % nx, nx, xs);
      axis3((i / nx) % ny, ny, ys);
      axis3(i / (nx * ny), nz, zs);
      pull_density(pop, pop_geo(nx, ny, nz), xs, ys, zs, nx, lb, ra, rb);
    }
    rho[i] = ra;
    rho[(size_t)N + i] = rb;
  }
}

template <typename real>
__global__ void k_fill(real* __restrict__ p, size_t n, real v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ----------------------------------------------------------------------------
// Host launchers
static int grid_for(size_t n, int block) {
  size_t g = (n + block - 1) / block;
  return (int)(g > 8192 ? 8192 : (g < 1 ? 1 : g));
}

hipError_t launch_links(const uint8_t* solid, uint32_t* links, int nx, int ny, int nz,
                        hipStream_t s) {
  size_t N = (size_t)nx * ny * nz;
  hipLaunchKernelGGL(k_links, dim3(grid_for(N, 256)), dim3(256), 0, s, solid, links, nx, ny, nz);
  return hipGetLastError();
}

hipError_t launch_init(int dtype, void* pop, const double* ra, const double* rb,
                       const uint32_t* links, int nx, int ny, int nz, hipStream_t s) {
  const int N = nx * ny * nz, P = nx * ny;
  const PopGeo g = pop_geo(nx, ny, nz);
  if (dtype == 0)
    hipLaunchKernelGGL(k_init<double>, dim3(grid_for(N, 256)), dim3(256), 0, s, (double*)pop, ra,
                       rb, links, N, P, g);
  else
    hipLaunchKernelGGL(k_init<float>, dim3(grid_for(N, 256)), dim3(256), 0, s, (float*)pop, ra, rb,
                       links, N, P, g);
  return hipGetLastError();
}

hipError_t launch_pop_repack(int dtype, const void* src, void* dst, int nx, int ny, int nz,
                             bool to_blocked, hipStream_t s) {
  const int N = nx * ny * nz, P = nx * ny;
  const PopGeo g = pop_geo(nx, ny, nz);
  const size_t total = (size_t)2 * Q * N;
  const size_t gb = (total + 255) / 256;
  const unsigned grid = (unsigned)(gb > 65536 ? 65536 : gb);
#define SCD_REPACK(T)                                                                            \
  if (to_blocked)                                                                                \
    hipLaunchKernelGGL((k_pop_repack<T, true>), dim3(grid), dim3(256), 0, s, (const T*)src,       \
                       (T*)dst, N, P, g);                                                        \
  else                                                                                           \
    hipLaunchKernelGGL((k_pop_repack<T, false>), dim3(grid), dim3(256), 0, s, (const T*)src,      \
                       (T*)dst, N, P, g);
  if (dtype == 0) {
    SCD_REPACK(double)
  } else {
    SCD_REPACK(float)
  }
#undef SCD_REPACK
  return hipGetLastError();
}

hipError_t launch_density(int dtype, const void* pop, const uint32_t* links, double* rho, int nx,
                          int ny, int nz, hipStream_t s) {
  const int N = nx * ny * nz, P = nx * ny;
  const PopGeo g = pop_geo(nx, ny, nz);
  if (dtype == 0)
    hipLaunchKernelGGL(k_density<double>, dim3(grid_for(N, 256)), dim3(256), 0, s,
                       (const double*)pop, links, rho, N, P, g);
  else
    hipLaunchKernelGGL(k_density<float>, dim3(grid_for(N, 256)), dim3(256), 0, s,
                       (const float*)pop, links, rho, N, P, g);
  return hipGetLastError();
}

hipError_t launch_stream_density(int dtype, const void* pop, const uint32_t* links, void* rho,
                                 int nx, int ny, int nz, hipStream_t s) {
  size_t N = (size_t)nx * ny * nz;
  if (dtype == 0)
    hipLaunchKernelGGL(k_stream_density<double>, dim3(grid_for(N, 256)), dim3(256), 0, s,
                       (const double*)pop, links, (double*)rho, nx, ny, nz);
  else
    hipLaunchKernelGGL(k_stream_density<float>, dim3(grid_for(N, 256)), dim3(256), 0, s,
                       (const float*)pop, links, (float*)rho, nx, ny, nz);
  return hipGetLastError();
}

hipError_t launch_fill(int dtype, void* p, size_t n, double v, hipStream_t s) {
  if (dtype == 0)
    hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, (double*)p, n, v);
  else
    hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, (float*)p, n,
                       (float)v);
  return hipGetLastError();
}

// Compiled variants (tx, ty, var, wpe): tile shape, z-march variant and
// the minimum waves per SIMD the register allocation must allow.
#define SCD_VARIANTS(X)                                                                   \
  X(64, 4, 0, 1) X(32, 8, 0, 1) X(64, 4, 1, 1) X(32, 4, 2, 2) X(32, 8, 2, 2) X(32, 4, 3, 2) \
  X(64, 4, 3, 2) X(32, 8, 3, 2) X(32, 4, 4, 1) X(32, 4, 5, 1) X(32, 4, 5, 2) X(32, 8, 5, 2) \
  X(64, 4, 5, 2) X(32, 8, 6, 2) X(32, 4, 6, 1) X(64, 4, 6, 2) X(32, 4, 7, 1) X(64, 4, 7, 2) \
  X(32, 4, 8, 1) X(32, 8, 9, 1) X(32, 8, 10, 1) X(64, 8, 9, 2) X(64, 8, 10, 2) X(32, 16, 11, 1)

static const int kVariants[][4] = {
#define SCD_ROW(a, b, v, w) {a, b, v, w},
    SCD_VARIANTS(SCD_ROW)
#undef SCD_ROW
};

int variant_count() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }
void variant_at(int i, int* tx, int* ty, int* var, int* wpe) {
  *tx = kVariants[i][0];
  *ty = kVariants[i][1];
  *var = kVariants[i][2];
  *wpe = kVariants[i][3];
}
int variant_find(int tx, int ty, int var, int wpe) {
  for (int i = 0; i < variant_count(); ++i)
    if (kVariants[i][0] == tx && kVariants[i][1] == ty && kVariants[i][2] == var &&
        kVariants[i][3] == wpe)
      return i;
  return -1;
}

template <typename real>
static hipError_t launch_step_t(const LatDev<real>& L, int variant, int zc, int remap,
                                hipStream_t s) {
  if (variant < 0 || variant >= variant_count()) return hipErrorInvalidValue;
  const int tx = kVariants[variant][0], ty = kVariants[variant][1];
  const int var = kVariants[variant][2], wpe = kVariants[variant][3];
  const int gx = (L.nx + tx - 1) / tx, gy = (L.ny + ty - 1) / ty;
  const int nch = (L.nz + zc - 1) / zc;
  const int total = gx * gy * nch;
  const int blocks = remap ? ((total + 7) / 8) * 8 : total;
#define SCD_LAUNCH(a, b, v, w)                                                              \
  if (tx == a && ty == b && var == v && wpe == w) {                                         \
    hipLaunchKernelGGL((k_step<real, a, b, v, w>), dim3(blocks),                            \
                       dim3(StepShape<real, a, b, v>::THREADS), 0, s, L, gx, gy, nch, zc, remap); \
    return hipGetLastError();                                                               \
  }
  SCD_VARIANTS(SCD_LAUNCH)
#undef SCD_LAUNCH
  return hipErrorInvalidValue;
}

hipError_t launch_step(int dtype, const void* src, void* dst, const uint32_t* links, int nx,
                       int ny, int nz, const PhysD& ph, int variant, int zc, int remap,
                       hipStream_t s, void* mom_out) {
  if (dtype == 0) {
    LatDev<double> L{(const double*)src, (double*)dst, links, nx, ny, nz, nx * ny * nz,
                     pop_geo(nx, ny, nz), phys_cast<double>(ph), (double*)mom_out};
    return launch_step_t(L, variant, zc, remap, s);
  }
  LatDev<float> L{(const float*)src, (float*)dst, links, nx, ny, nz, nx * ny * nz,
                  pop_geo(nx, ny, nz), phys_cast<float>(ph), (float*)mom_out};
  return launch_step_t(L, variant, zc, remap, s);
}

bool variant_writes_moments(int variant) {
  if (variant < 0 || variant >= variant_count()) return false;
  const int var = kVariants[variant][2];
  return var == VAR_DUAL || var == VAR_TRIPLE || var == VAR_QUAD || var == VAR_ROWS2 ||
         var == VAR_ROWS1 || var == VAR_ROWS4;
}

template <typename real>
static hipError_t launch_batch_t(const void* h_descs, int ndesc, const int* h_geo, int grid,
                                 int variant, int remap, hipStream_t s) {
  if (variant < 0 || variant >= variant_count()) return hipErrorInvalidValue;
  if (ndesc < 1 || ndesc > BATCH_DESC_MAX) return hipErrorInvalidValue;
  BatchDescs<real> D;
  std::memset(&D, 0, sizeof(D));
  std::memcpy(D.L, h_descs, (size_t)ndesc * sizeof(LatDev<real>));
  D.n = ndesc;
  D.start[0] = 0;
  for (int m = 0; m < ndesc; ++m) {
    const int gx = h_geo[3 * m], gz = h_geo[3 * m + 1], zc = h_geo[3 * m + 2];
    const LatDev<real>& L = D.L[m];
    const int gy = (L.ny + kVariants[variant][1] - 1) / kVariants[variant][1];
    if (gx < 1 || gz < 1 || zc < 1 || gz != (L.nz + zc - 1) / zc) return hipErrorInvalidValue;
    D.gx[m] = gx;
    D.gz[m] = gz;
    D.zc[m] = zc;
    D.start[m + 1] = D.start[m] + gx * gy * gz;
  }
  const int tx = kVariants[variant][0], ty = kVariants[variant][1];
  const int var = kVariants[variant][2], wpe = kVariants[variant][3];
#define SCD_LAUNCHB(a, b, v, w)                                                                 \
  if (tx == a && ty == b && var == v && wpe == w) {                                             \
    hipLaunchKernelGGL((k_step_batch<real, a, b, v, w>), dim3(grid),                            \
                       dim3(StepShape<real, a, b, v>::THREADS), 0, s, D, remap);                \
    return hipGetLastError();                                                                   \
  }
  SCD_VARIANTS(SCD_LAUNCHB)
#undef SCD_LAUNCHB
  return hipErrorInvalidValue;
}

hipError_t launch_step_batch(int dtype, const void* h_descs, int ndesc, const int* h_geo, int grid,
                             int variant, int remap, hipStream_t s) {
  if (dtype == 0) return launch_batch_t<double>(h_descs, ndesc, h_geo, grid, variant, remap, s);
  return launch_batch_t<float>(h_descs, ndesc, h_geo, grid, variant, remap, s);
}

size_t latdev_size(int dtype) { return dtype == 0 ? sizeof(LatDev<double>) : sizeof(LatDev<float>); }

void latdev_fill(int dtype, void* out, const void* src, void* dst, const uint32_t* links, int nx,
                 int ny, int nz, const PhysD& ph) {
  if (dtype == 0) {
    LatDev<double> L{(const double*)src, (double*)dst, links, nx, ny, nz, nx * ny * nz,
                     pop_geo(nx, ny, nz), phys_cast<double>(ph), nullptr};
    *(LatDev<double>*)out = L;
  } else {
    LatDev<float> L{(const float*)src, (float*)dst, links, nx, ny, nz, nx * ny * nz,
                    pop_geo(nx, ny, nz), phys_cast<float>(ph), nullptr};
    *(LatDev<float>*)out = L;
  }
}

}  // namespace scd
