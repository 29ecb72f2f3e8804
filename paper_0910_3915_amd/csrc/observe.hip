// observe.hip -- global reductions and the contact-angle observable on gfx950.
//
// Reductions accumulate in FP64 for both state precisions: a grid-stride
// pass per thread, a wavefront butterfly (__shfl_xor, lowered to DPP / LDS
// permutes), a cross-wave step in LDS, per-block partials, and a one-block
// finish that adds the partials in a fixed order, so results are
// bit-reproducible run to run.
//
// Contact angle (Sec. 3, Eq. geoCA): the order parameter phi = rho_A - rho_B
// (Sec. 2) is evaluated on the reference layer, on the first fluid layer and
// on the droplet's column; a one-block kernel then measures the cap with two
// estimators:
//   E1 -- zero crossings of phi by linear interpolation: apex height on the
//         column, four half-chords in the reference layer, sphere radius
//         R = (aref^2 + H^2) / 2H through the reference circle and the apex,
//         base half-width a^2 = 2Rh - h^2 at the wall, theta = 2 atan(h / a);
//   E2 -- the same geometry from sums of a smoothed indicator
//         chi = S((phi + eps) / 2 eps), S(t) = 3t^2 - 2t^3 on [0, 1]: the
//         column height H = chi(kref)/2 + sum of chi above it up to the top of
//         the droplet, the reference area sum(chi) = pi aref^2.  E2 is a
//         smooth function of the state and seeds the adjoint.
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"

namespace scd {

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* sh) {
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
  __syncthreads();
}

template <typename real>
__global__ __launch_bounds__(256) void k_obs_partial(const real* __restrict__ pop,
                                                     const uint32_t* __restrict__ links, int N,
                                                     int P, PopGeo g,
                                                     double* __restrict__ partials) {
  __shared__ double sh[6 * 16];
  double v[6] = {0, 0, 0, 0, 0, 0};  // mass A, mass B, Px, Py, Pz, non-finite count
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    if (links[i] & SELF_SOLID) continue;
    const size_t si = pop_slot_i(g, i, P);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const double a = (double)pop[si + k * PBLK];
      const double b = (double)pop[g.sp + si + k * PBLK];
      if (!isfinite(a) || !isfinite(b)) v[5] += 1.0;
      v[0] += a;
      v[1] += b;
      const double ab = a + b;
      if (CX[k]) v[2] += CX[k] * ab;
      if (CY[k]) v[3] += CY[k] * ab;
      if (CZ[k]) v[4] += CZ[k] * ab;
    }
  }
  block_sum<6>(v, sh);
  if (threadIdx.x == 0)
    for (int j = 0; j < 6; ++j) partials[blockIdx.x * RED_STRIDE + j] = v[j];
}

// one block: partials of nblocks blocks -> result[0..5]
__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ partials,
                                                      int nblocks, int nvals,
                                                      double* __restrict__ result) {
  __shared__ double sh[8 * 16];
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
    for (int j = 0; j < nvals; ++j) v[j] += partials[b * RED_STRIDE + j];
  block_sum<8>(v, sh);
  if (threadIdx.x == 0)
    for (int j = 0; j < nvals; ++j) result[j] = v[j];
}

hipError_t launch_observables(int dtype, const void* pop, const uint32_t* links, int nx, int ny,
                              int nz, double* partials, double* result, hipStream_t s) {
  const int N = nx * ny * nz, P = nx * ny;
  const PopGeo g = pop_geo(nx, ny, nz);
  if (dtype == 0)
    hipLaunchKernelGGL(k_obs_partial<double>, dim3(RED_BLOCKS), dim3(256), 0, s,
                       (const double*)pop, links, N, P, g, partials);
  else
    hipLaunchKernelGGL(k_obs_partial<float>, dim3(RED_BLOCKS), dim3(256), 0, s,
                       (const float*)pop, links, N, P, g, partials);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, partials, RED_BLOCKS, 6, result);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Contact angle
// phi scratch layout (doubles): [0, A) reference layer, [A, 2A) first fluid
// layer, [2A, 2A + nz) column, A = nx * ny.  Wall nodes hold 0.
template <typename real>
__global__ void k_ca_phi(const real* __restrict__ pop, const uint32_t* __restrict__ links, int nx,
                         int ny, int nz, CaDev c, double* __restrict__ phi) {
  const int A = nx * ny;
  const int total = 2 * A + nz;
  const PopGeo g = pop_geo(nx, ny, nz);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
    int x, y, z;
    if (t < A) { x = t % nx; y = t / nx; z = c.zs + c.off; }
    else if (t < 2 * A) { x = (t - A) % nx; y = (t - A) / nx; z = c.zs + 1; }
    else { x = c.ic; y = c.jc; z = t - 2 * A; }
    double v = 0;
    if (z >= 0 && z < nz) {
      const int i = (z * ny + y) * nx + x;
      if (!(links[i] & SELF_SOLID)) {
        double ra = 0, rb = 0;
        const size_t si = pop_slot(g, z, y * nx + x);
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          ra += (double)pop[si + k * PBLK];
          rb += (double)pop[g.sp + si + k * PBLK];
        }
        v = ra - rb;  // order parameter (Sec. 2)
      }
    }
    phi[t] = v;
  }
}

__device__ __forceinline__ double smoothstep(double t) {
  return t <= 0.0 ? 0.0 : (t >= 1.0 ? 1.0 : t * t * (3.0 - 2.0 * t));
}
__device__ __forceinline__ double dsmoothstep(double t) {
  return (t <= 0.0 || t >= 1.0) ? 0.0 : 6.0 * t * (1.0 - t);
}

struct CaGeom {
  int nx, ny, nz;
  const uint32_t* links;
  CaDev c;
  __device__ bool solid(int x, int y, int z) const {
    if (z < 0 || z >= nz) return true;
    return links[(z * ny + y) * nx + x] & SELF_SOLID;
  }
};

// The column (ic, jc) and, per z-layer, its row y = jc and column x = ic:
// everything the serial scans below read, staged in LDS so that each scan
// step waits on LDS rather than on memory.
struct LayerRC {
  const double* row;  // phi(x, jc), x = 0 .. nx - 1
  const double* col;  // phi(ic, y), y = 0 .. ny - 1
  int jc;
  __device__ double at(int x, int y) const { return y == jc ? row[x] : col[y]; }
};

// first crossing > 0 -> <= 0 of the column above k0 (colsolid: 1 at walls),
// NaN if none
__device__ double col_crossing(const CaGeom& g, const double* col, const double* colsolid,
                               int k0) {
  for (int k = k0; k + 1 < g.nz; ++k) {
    if (colsolid[k + 1] != 0.0) break;
    const double p0 = col[k], p1 = col[k + 1];
    if (p0 > 0.0 && p1 <= 0.0) return k + p0 / (p0 - p1);
  }
  return __builtin_nan("");
}

// Half-chord along (sx, sy) from the droplet axis: the first crossing
// > 0 -> <= 0 of phi between neighbouring nodes of the ray, which steps
// periodically (the coordinates advance by one with wrap-around, no modulo).
__device__ double layer_ray(const CaGeom& g, const LayerRC& layer, int sx, int sy, int* flags) {
  const int len = sx != 0 ? g.nx : g.ny;
  int x = wrap_index(g.c.ic, g.nx), y = wrap_index(g.c.jc, g.ny);
  double p0 = layer.at(x, y);
  for (int m = 0; m < len / 2; ++m) {
    x += sx;
    y += sy;
    if (x == g.nx) x = 0;
    if (x < 0) x = g.nx - 1;
    if (y == g.ny) y = 0;
    if (y < 0) y = g.ny - 1;
    const double p1 = layer.at(x, y);
    if (p0 > 0.0 && p1 <= 0.0) return m + p0 / (p0 - p1);
    p0 = p1;
  }
  *flags |= 8;  // SCD_CA_RAY_LIMIT
  return (double)(len / 2);
}

__device__ double mean_ray(const CaGeom& g, const LayerRC& layer, int* flags) {
  return 0.25 * (layer_ray(g, layer, 1, 0, flags) + layer_ray(g, layer, -1, 0, flags) +
                 layer_ray(g, layer, 0, 1, flags) + layer_ray(g, layer, 0, -1, flags));
}

constexpr double RAD2DEG = 57.295779513082320876798154814105;

// sphere through the reference circle (aref2 = aref^2) and the apex H above
// it; base half-width at the wall from the cap height h
__device__ double cap_theta(double aref2, double H, double h, double* R, double* a, int* flat) {
  *R = (aref2 + H * H) / (2.0 * H);
  const double a2 = 2.0 * (*R) * h - h * h;
  if (!(a2 > 0.0)) { *flat = 1; *a = 0.0; return 180.0; }
  *flat = 0;
  *a = sqrt(a2);
  return 2.0 * atan2(h, *a) * RAD2DEG;
}

// result slots
enum {
  R_TH1 = 0, R_H1, R_A1, R_R1, R_AREF1, R_BH1,
  R_TH2, R_H2, R_A2, R_R2, R_AREF2, R_BH2,
  R_CX, R_CY, R_FLAGS, R_STATUS, R_DTH_DH, R_DTH_DA, R_KEND, R_RCUT
};

// Radius of the disk around the column over which E2 sums the reference
// layer: the largest of the four half-chords plus 4 lattice units (the
// indicator's transition band), so that A-rich regions of the layer that are
// not this droplet (a wall film, a second droplet) are left out.  Infinite
// (whole layer) when phi <= 0 on the column at the reference layer.
__device__ double e2_window(const CaGeom& g, const LayerRC& ref) {
  if (!(ref.at(g.c.ic, g.c.jc) > 0.0)) return __builtin_inf();
  int f = 0;
  double r = layer_ray(g, ref, 1, 0, &f);
  r = fmax(r, layer_ray(g, ref, -1, 0, &f));
  r = fmax(r, layer_ray(g, ref, 0, 1, &f));
  r = fmax(r, layer_ray(g, ref, 0, -1, &f));
  return r + 4.0;
}

// periodic (minimum image) distance along one axis
__device__ __forceinline__ int image_dist(int a, int b, int n) {
  const int d = a > b ? a - b : b - a;
  return d < n - d ? d : n - d;
}

__device__ __forceinline__ bool in_window(const CaGeom& g, double rcut, int x, int y) {
  const double dx = image_dist(x, g.c.ic, g.nx), dy = image_dist(y, g.c.jc, g.ny);
  return dx * dx + dy * dy <= rcut * rcut;
}

// Layer sums of the reference layer (sum of chi inside the E2 window; sum of
// x, y and count where phi > 0), split over CA_LAYER_BLOCKS workgroups with
// one node per thread.  Each workgroup stages the layer's row and column
// through the droplet axis and finds the E2 window itself, then writes its
// four partial sums to part; workgroup 0 also writes the window radius to
// part[4 * CA_LAYER_BLOCKS].
constexpr int CA_LAYER_BLOCKS = 64;  // one wavefront of k_ca_finish adds them
__global__ __launch_bounds__(256) void k_ca_layer(const uint32_t* __restrict__ links, int nx,
                                                  int ny, int nz, CaDev c,
                                                  const double* __restrict__ phi,
                                                  double* __restrict__ part) {
  __shared__ double sh[4 * 16];
  extern __shared__ double stage[];  // 8 * (nx + ny) bytes
  const CaGeom g{nx, ny, nz, links, c};
  const int A = nx * ny;
  const int kref = c.zs + c.off;
  const double* ref = phi;
  double* rowR = stage;
  double* colR = rowR + nx;
  for (int t = threadIdx.x; t < nx; t += blockDim.x) rowR[t] = ref[c.jc * nx + t];
  for (int t = threadIdx.x; t < ny; t += blockDim.x) colR[t] = ref[t * nx + c.ic];
  __syncthreads();
  const LayerRC refRC{rowR, colR, c.jc};
  if (threadIdx.x == 0) sh[0] = e2_window(g, refRC);
  __syncthreads();
  const double rcut = sh[0];
  __syncthreads();
  double v[4] = {0, 0, 0, 0};
  const bool layer_in = kref >= 0 && kref < nz;
  const uint32_t* lref = links + (size_t)(layer_in ? kref : 0) * A;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < A; t += gridDim.x * blockDim.x) {
    if (!layer_in || (lref[t] & SELF_SOLID)) continue;
    const int y = t / nx, x = t - y * nx;
    const double p = ref[t];
    if (in_window(g, rcut, x, y)) v[0] += smoothstep((p + c.eps) / (2.0 * c.eps));
    if (p > 0.0) { v[1] += x; v[2] += y; v[3] += 1.0; }
  }
  block_sum<4>(v, sh);
  if (threadIdx.x == 0) {
    for (int j = 0; j < 4; ++j) part[4 * blockIdx.x + j] = v[j];
    if (blockIdx.x == 0) part[4 * CA_LAYER_BLOCKS] = rcut;
  }
}

__global__ __launch_bounds__(256) void k_ca_finish(const uint32_t* __restrict__ links, int nx,
                                                   int ny, int nz, CaDev c,
                                                   const double* __restrict__ phi,
                                                   const double* __restrict__ part,
                                                   double* __restrict__ res) {
  extern __shared__ double stage[];  // ca_stage_bytes(nx, ny, nz)
  const CaGeom g{nx, ny, nz, links, c};
  const int A = nx * ny;
  const int kref = c.zs + c.off;
  const double* ref = phi;
  const double* low = phi + A;
  double* rowR = stage;
  double* colR = rowR + nx;
  double* rowL = colR + ny;
  double* colL = rowL + nx;
  double* col = colL + ny;
  double* colsolid = col + nz;
  for (int t = threadIdx.x; t < nx; t += blockDim.x) {
    rowR[t] = ref[c.jc * nx + t];
    rowL[t] = low[c.jc * nx + t];
  }
  for (int t = threadIdx.x; t < ny; t += blockDim.x) {
    colR[t] = ref[t * nx + c.ic];
    colL[t] = low[t * nx + c.ic];
  }
  for (int t = threadIdx.x; t < nz; t += blockDim.x) {
    col[t] = phi[2 * A + t];
    colsolid[t] = g.solid(c.ic, c.jc, t) ? 1.0 : 0.0;
  }
  __syncthreads();
  const LayerRC refRC{rowR, colR, c.jc}, lowRC{rowL, colL, c.jc};
  // the layer sums of k_ca_layer: lane b of the first wave takes workgroup
  // b's partials, and a fixed butterfly adds them
  static_assert(CA_LAYER_BLOCKS == 64, "one partial per lane of a wavefront");
  double v[4] = {0, 0, 0, 0};
  if (threadIdx.x < 64) {
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = part[4 * threadIdx.x + j];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      for (int off = 32; off > 0; off >>= 1) v[j] += __shfl_xor(v[j], off, 64);
  }
  if (threadIdx.x != 0) return;
  const double rcut = part[4 * CA_LAYER_BLOCKS];

  const double nan = __builtin_nan("");
  int flags = 0;
  double out[R_RCUT + 1];
  for (int j = 0; j <= R_RCUT; ++j) out[j] = 0.0;
  out[R_RCUT] = rcut;
  out[R_CX] = v[3] > 0.0 ? v[1] / v[3] : nan;
  out[R_CY] = v[3] > 0.0 ? v[2] / v[3] : nan;
  const double zw = c.zs + 0.5, d = kref - zw;
  double status = 0.0;
  if (!(col[c.zs + 1] > 0.0)) {
    flags |= 32;  // SCD_CA_NO_DROP
    out[R_TH1] = out[R_TH2] = nan;
    status = -4.0;
  } else {
    int flat = 0;
    if (col[kref] > 0.0) {
      const double ztop = col_crossing(g, col, colsolid, kref);
      if (isnan(ztop)) {
        flags |= 16;
        out[R_TH1] = nan;
      } else {
        const double h = ztop - zw, H = ztop - kref;
        const double aref = mean_ray(g, refRC, &flags);
        double R, a;
        out[R_TH1] = cap_theta(aref * aref, H, h, &R, &a, &flat);
        if (flat) flags |= 2;
        out[R_H1] = h; out[R_BH1] = H; out[R_AREF1] = aref; out[R_R1] = R; out[R_A1] = a;
      }
    } else {
      flags |= 1;  // SCD_CA_NO_REF
      const double ztop = col_crossing(g, col, colsolid, c.zs + 1);
      if (isnan(ztop)) {
        flags |= 16;
        out[R_TH1] = nan;
      } else {
        const double h = ztop - zw;
        const double a = mean_ray(g, lowRC, &flags);
        out[R_TH1] = 2.0 * atan2(h, a) * RAD2DEG;
        out[R_H1] = h; out[R_A1] = a; out[R_BH1] = ztop - kref; out[R_AREF1] = nan;
        out[R_R1] = (a * a + h * h) / (2.0 * h);
      }
    }
    // E2
    if (isinf(rcut)) flags |= 128;  // SCD_CA_E2_WHOLE_LAYER
    auto chi = [&](int k) {
      if (colsolid[k] != 0.0) return 0.0;
      return smoothstep((col[k] + c.eps) / (2.0 * c.eps));
    };
    int kend = kref + 1;
    while (kend < nz && chi(kend) > 0.0) ++kend;
    double H = 0.5 * chi(kref);
    for (int k = kref + 1; k < kend; ++k) H += chi(k);
    const double Aref = v[0] / M_PI;
    out[R_BH2] = H;
    out[R_AREF2] = sqrt(Aref);
    out[R_KEND] = kend;
    if (!(H > 0.0)) {
      flags |= 64;
      out[R_TH2] = nan;
    } else {
      const double h = H + d;
      double R, a;
      out[R_TH2] = cap_theta(Aref, H, h, &R, &a, &flat);
      if (flat) flags |= 4;
      out[R_H2] = h; out[R_R2] = R; out[R_A2] = a;
      if (!flat) {
        // partial derivatives of theta_E2 (radians) with respect to H and to
        // Aref = aref^2, from a^2 = (Aref + H^2) h / H - h^2, h = H + d
        const double a2 = a * a;
        const double da2_dA = h / H;
        const double da2_dH =
            ((2.0 * H * h + (Aref + H * H)) * H - (Aref + H * H) * h) / (H * H) - 2.0 * h;
        const double den = a2 + h * h;
        out[R_DTH_DH] = 2.0 * (a - h * da2_dH / (2.0 * a)) / den;
        out[R_DTH_DA] = 2.0 * (-h * da2_dA / (2.0 * a)) / den;
      }
    }
  }
  out[R_FLAGS] = flags;
  out[R_STATUS] = status;
  for (int j = 0; j <= R_RCUT; ++j) res[j] = out[j];
}

hipError_t launch_contact_angle(int dtype, const void* pop, const uint32_t* links, int nx, int ny,
                                int nz, CaDev cfg, double* phi_scratch, double* partials,
                                double* result, hipStream_t s) {
  const int total = 2 * nx * ny + nz;
  const int blocks = (total + 255) / 256;
  if (dtype == 0)
    hipLaunchKernelGGL(k_ca_phi<double>, dim3(blocks), dim3(256), 0, s, (const double*)pop, links,
                       nx, ny, nz, cfg, phi_scratch);
  else
    hipLaunchKernelGGL(k_ca_phi<float>, dim3(blocks), dim3(256), 0, s, (const float*)pop, links,
                       nx, ny, nz, cfg, phi_scratch);
  const size_t stage = (size_t)8 * (2 * (size_t)nx + 2 * (size_t)ny + 2 * (size_t)nz);
  if (stage > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_ca_finish,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)stage);
    if (e != hipSuccess) return e;
  }
  const size_t lstage = (size_t)8 * ((size_t)nx + (size_t)ny);
  if (lstage > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_ca_layer,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lstage);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_ca_layer, dim3(CA_LAYER_BLOCKS), dim3(256), lstage, s, links, nx, ny, nz,
                     cfg, phi_scratch, partials);
  hipLaunchKernelGGL(k_ca_finish, dim3(1), dim3(256), stage, s, links, nx, ny, nz, cfg,
                     phi_scratch, partials, result);
  return hipGetLastError();
}

// Scratch of the contact angle in a file-scope device array, for callers
// that allocate nothing (scd_contact_angle_static): the phi layers and column
// (CA_STATIC_PHI doubles at most), the layer partials and the result slots.
// Each GPU holds its own copy for the life of the process; host code uses
// the address hipGetSymbolAddress returns for the current device, never the
// array's name.
constexpr size_t CA_STATIC_PHI = 2 * CA_STATIC_MAX_PLANE + CA_STATIC_MAX_NZ;
constexpr size_t CA_STATIC_PART = 512;  // >= 4 * CA_LAYER_BLOCKS + 1
static_assert(4 * CA_LAYER_BLOCKS + 1 <= CA_STATIC_PART, "layer partials");
static __device__ __align__(256) double scratch[CA_STATIC_PHI + CA_STATIC_PART + CA_SLOTS];

hipError_t ca_static_scratch(double** phi, double** partials, double** result) {
  constexpr int MAX_DEV = 64;
  static std::mutex lock;
  static void* addr[MAX_DEV] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEV) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(lock);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  double* base = static_cast<double*>(addr[dev]);
  *phi = base;
  *partials = base + CA_STATIC_PHI;
  *result = base + CA_STATIC_PHI + CA_STATIC_PART;
  return hipSuccess;
}

// Seed of the adjoint: lambda_k^A = dL/dtheta * dtheta/dphi, lambda_k^B =
// -lambda_k^A at every node of the reference layer and of the column run of
// the droplet above it (all other entries are zeroed beforehand).
template <typename real>
__global__ void k_ca_seed(const uint32_t* __restrict__ links, int nx, int ny, int nz, CaDev c,
                          const double* __restrict__ phi, const double* __restrict__ res,
                          double dL, real* __restrict__ lam) {
  const int A = nx * ny;
  const PopGeo pg = pop_geo(nx, ny, nz);
  const int kref = c.zs + c.off;
  const int kend = (int)res[R_KEND];
  const double dH = res[R_DTH_DH], dA = res[R_DTH_DA];
  const CaGeom g{nx, ny, nz, links, c};
  const double rcut = res[R_RCUT];
  const int total = A + nz;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
    int x, y, z;
    double p;
    if (t < A) { x = t % nx; y = t / nx; z = kref; p = phi[t]; }
    else { x = c.ic; y = c.jc; z = t - A; p = phi[2 * A + z]; if (z <= kref || z >= kend) continue; }
    const int i = (z * ny + y) * nx + x;
    if (links[i] & SELF_SOLID) continue;
    const double dchi = dsmoothstep((p + c.eps) / (2.0 * c.eps)) / (2.0 * c.eps);
    double gr;
    if (t < A) {
      gr = in_window(g, rcut, x, y) ? dA * dchi / M_PI : 0.0;
      if (x == c.ic && y == c.jc) gr += 0.5 * dH * dchi;
    } else {
      gr = dH * dchi;
    }
    const real va = (real)(dL * gr), vb = (real)(-dL * gr);
    const size_t si = pop_slot(pg, z, y * nx + x);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      lam[si + k * PBLK] = va;
      lam[pg.sp + si + k * PBLK] = vb;
    }
  }
}

hipError_t launch_ca_seed(int dtype, const uint32_t* links, int nx, int ny, int nz, CaDev cfg,
                          const double* phi_scratch, const double* result, double dL_dtheta,
                          void* lambda, hipStream_t s) {
  hipError_t e = launch_fill(dtype, lambda, 2 * (size_t)pop_geo(nx, ny, nz).sp, 0.0, s);
  if (e != hipSuccess) return e;
  const int total = nx * ny + nz;
  const int blocks = (total + 255) / 256;
  if (dtype == 0)
    hipLaunchKernelGGL(k_ca_seed<double>, dim3(blocks), dim3(256), 0, s, links, nx, ny, nz, cfg,
                       phi_scratch, result, dL_dtheta, (double*)lambda);
  else
    hipLaunchKernelGGL(k_ca_seed<float>, dim3(blocks), dim3(256), 0, s, links, nx, ny, nz, cfg,
                       phi_scratch, result, dL_dtheta, (float*)lambda);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Pressure tensor (Sec. 4.1) at every node from the post-stream populations
// of the current state; rho: their densities at every node (2 N values).
// At a fluid node
//   P_ij = sum_a sum_k (c_ki - u_i)(c_kj - u_j) n_k^a
//        + 1/2 sum_k W_k c_ki c_kj [psi^A G^A(y) psi^B(y) + psi^B G^B(y) psi^A(y)]
// with y = x + c_k and u the velocity of the fluid, (sum_a j^a + F / 2) /
// sum_a rho^a (F the total Shan-Chen and wall force of the node, from the
// same neighbour sums); the paper's sum over the two ordered species pairs
// with prefactor 1/4 gives the 1/2, its pair factor is the dyad of (x - x'),
// and wall neighbours carry their content and g_wall^a as in the force.  At a
// wall node (the wall taken as a component) there is no kinetic part and the
// tensor is the wall's half of each wall-fluid pair,
//   1/2 sum_{k: y fluid} W_k c_ki c_kj [g_wall^A psi^A(y) psi_w^B + g_wall^B psi^B(y) psi_w^A].
// Output P[c * N + i] (FP64), c = xx, yy, zz, xy, xz, yz.
template <typename real>
__global__ __launch_bounds__(256) void k_pressure(const real* __restrict__ pop,
                                                  const uint32_t* __restrict__ links,
                                                  const real* __restrict__ rho, int nx, int ny,
                                                  int nz, Phys<real> ph, double* __restrict__ P) {
  const int N = nx * ny * nz;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    const uint32_t lb = links[i];
    double out[6] = {0, 0, 0, 0, 0, 0};
    int xs[3], ys[3], zs[3];
    axis3(i % nx, nx, xs);
    axis3((i / nx) % ny, ny, ys);
    axis3(i / (nx * ny), nz, zs);
    if (lb & SELF_SOLID) {
      const double wA = (double)ph.gw[0] * (double)ph.psiw[1];  // felt by A from this wall node
      const double wB = (double)ph.gw[1] * (double)ph.psiw[0];
#pragma unroll
      for (int k = 1; k < Q; ++k) {
        if ((lb >> k) & 1u) continue;  // wall-wall pairs carry no force
        const int y = nbr_index(xs, ys, zs, nx, ny, CX[k], CY[k], CZ[k]);
        const double qA = psi_of(ph.psi_form, (double)rho[y]);
        const double qB = psi_of(ph.psi_form, (double)rho[(size_t)N + y]);
        const double w = (CX[k] * CX[k] + CY[k] * CY[k] + CZ[k] * CZ[k]) == 1 ? ph.wa : ph.wd;
        const double br = 0.5 * w * (wA * qA + wB * qB);
        out[0] += CX[k] * CX[k] * br; out[1] += CY[k] * CY[k] * br; out[2] += CZ[k] * CZ[k] * br;
        out[3] += CX[k] * CY[k] * br; out[4] += CX[k] * CZ[k] * br; out[5] += CY[k] * CZ[k] * br;
      }
    } else {
      real n[38];
      pull38(pop, pop_geo(nx, ny, nz), xs, ys, zs, nx, lb, n);
      const double pA = psi_of(ph.psi_form, (double)rho[i]);
      const double pB = psi_of(ph.psi_form, (double)rho[(size_t)N + i]);
      // pair terms and the force sums S^a = sum_k W_k G^a psi^b(y) c_k
      double t[6] = {0, 0, 0, 0, 0, 0}, sA[3] = {0, 0, 0}, sB[3] = {0, 0, 0};
#pragma unroll
      for (int k = 1; k < Q; ++k) {
        const bool wall = (lb >> k) & 1u;
        double qA = ph.psiw[0], qB = ph.psiw[1], gA = ph.gw[0], gB = ph.gw[1];
        if (!wall) {
          const int y = nbr_index(xs, ys, zs, nx, ny, CX[k], CY[k], CZ[k]);
          qA = psi_of(ph.psi_form, (double)rho[y]);
          qB = psi_of(ph.psi_form, (double)rho[(size_t)N + y]);
          gA = gB = ph.gab;
        }
        const double w = (CX[k] * CX[k] + CY[k] * CY[k] + CZ[k] * CZ[k]) == 1 ? ph.wa : ph.wd;
        const double br = w * (pA * gA * qB + pB * gB * qA);
        t[0] += CX[k] * CX[k] * br; t[1] += CY[k] * CY[k] * br; t[2] += CZ[k] * CZ[k] * br;
        t[3] += CX[k] * CY[k] * br; t[4] += CX[k] * CZ[k] * br; t[5] += CY[k] * CZ[k] * br;
        const double eA = w * gA * qB, eB = w * gB * qA;
        sA[0] += CX[k] * eA; sA[1] += CY[k] * eA; sA[2] += CZ[k] * eA;
        sB[0] += CX[k] * eB; sB[1] += CY[k] * eB; sB[2] += CZ[k] * eB;
      }
      double R = 0, j[3] = {0, 0, 0}, m[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        const double f = (double)n[k] + (double)n[Q + k];
        R += f;
        j[0] += CX[k] * f; j[1] += CY[k] * f; j[2] += CZ[k] * f;
        m[0] += CX[k] * CX[k] * f; m[1] += CY[k] * CY[k] * f; m[2] += CZ[k] * CZ[k] * f;
        m[3] += CX[k] * CY[k] * f; m[4] += CX[k] * CZ[k] * f; m[5] += CY[k] * CZ[k] * f;
      }
      // F = F^A + F^B = -psi^A S^A - psi^B S^B; u = (J + F / 2) / R
      double u[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) u[d] = (j[d] + 0.5 * (-pA * sA[d] - pB * sB[d])) / R;
      // sum_k (c - u)_i (c - u)_j f = M_ij - u_i J_j - J_i u_j + R u_i u_j
      const int ci[6] = {0, 1, 2, 0, 0, 1}, cj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
      for (int c = 0; c < 6; ++c)
        out[c] = m[c] - u[ci[c]] * j[cj[c]] - j[ci[c]] * u[cj[c]] + R * u[ci[c]] * u[cj[c]] +
                 0.5 * t[c];
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) P[(size_t)c * N + i] = out[c];
  }
}

// One workgroup per plane z: mean over all its nodes (fluid and wall) of
// P_zz - (P_xx + P_yy) / 2, Eq. gammaMechDef's integrand for interfaces
// normal to z.
__global__ __launch_bounds__(256) void k_plane_tension(int nx, int ny, int nz,
                                                       const double* __restrict__ P,
                                                       double* __restrict__ profile) {
  __shared__ double sh[2 * 16];
  const int N = nx * ny * nz, A = nx * ny;
  const int z = blockIdx.x;
  double v[2] = {0, 0};
  for (int t = threadIdx.x; t < A; t += blockDim.x) {
    const int i = z * A + t;
    v[0] += P[(size_t)2 * N + i] - 0.5 * (P[i] + P[(size_t)N + i]);
    v[1] += 1.0;
  }
  block_sum<2>(v, sh);
  if (threadIdx.x == 0) profile[z] = v[0] / v[1];
}

// Radial decomposition about a centre c (Eq. mechRadGamma): per fluid node,
// with d = x - c (minimum image along the axes whose bit is set in periodic:
// bit 0 x, bit 1 y, bit 2 z; the plain difference along the others),
// P_N = d.P.d / |d|^2,
// P_T = (tr P - P_N) / 2 (the centre node itself adds 0), written over the
// tensor's first three components: P[i] = P_N - P_T, P[N + i] = phi,
// P[2N + i] = shell index b (b <= |d| < b + 1, from exact comparisons on
// |d|^2), or -1 for wall nodes and nodes beyond nbins shells.  Each thread
// reads all six components of its node before it writes any.
template <typename real>
__global__ __launch_bounds__(256) void k_radial_split(const real* __restrict__ pop,
                                                      const uint32_t* __restrict__ links,
                                                      int nx, int ny, int nz, double cx,
                                                      double cy, double cz, int nbins,
                                                      int periodic, double* __restrict__ P) {
  const int N = nx * ny * nz;
  auto image = [periodic](double d, int n, int axis) {
    if (!((periodic >> axis) & 1)) return d;
    if (d >= 0.5 * n) d -= n;
    if (d < -0.5 * n) d += n;
    return d;
  };
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    double v = 0.0, ph = 0.0, bin = -1.0;
    if (!(links[i] & SELF_SOLID)) {
      const double d0 = image((i % nx) - cx, nx, 0), d1 = image(((i / nx) % ny) - cy, ny, 1);
      const double d2 = image((i / (nx * ny)) - cz, nz, 2);
      const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
      int b = (int)floor(sqrt(r2));
      while ((double)(b + 1) * (b + 1) <= r2) ++b;
      while (b > 0 && (double)b * b > r2) --b;
      if (b < nbins) {
        bin = (double)b;
        if (r2 > 0.0) {
          const double p0 = P[i], p1 = P[(size_t)N + i], p2 = P[(size_t)2 * N + i];
          const double p3 = P[(size_t)3 * N + i], p4 = P[(size_t)4 * N + i];
          const double p5 = P[(size_t)5 * N + i];
          const double pn = (d0 * d0 * p0 + d1 * d1 * p1 + d2 * d2 * p2 +
                             2.0 * (d0 * d1 * p3 + d0 * d2 * p4 + d1 * d2 * p5)) / r2;
          v = pn - 0.5 * (p0 + p1 + p2 - pn);
        }
        double ra = 0, rb = 0;
        const PopGeo g = pop_geo(nx, ny, nz);
        const size_t si = pop_slot_i(g, i, nx * ny);
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          ra += (double)pop[si + k * PBLK];
          rb += (double)pop[g.sp + si + k * PBLK];
        }
        ph = ra - rb;
      }
    }
    P[i] = v;
    P[(size_t)N + i] = ph;
    P[(size_t)2 * N + i] = bin;
  }
}

// One workgroup per shell b: sums of P_N - P_T and of phi and the node count
// over the nodes of shell b, in a fixed order -> out[3 b .. 3 b + 2].
__global__ __launch_bounds__(256) void k_radial_shells(const double* __restrict__ P, int N,
                                                       double* __restrict__ out) {
  __shared__ double sh[3 * 16];
  const double b = (double)blockIdx.x;
  double v[3] = {0, 0, 0};
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    if (P[(size_t)2 * N + i] != b) continue;
    v[0] += P[i];
    v[1] += P[(size_t)N + i];
    v[2] += 1.0;
  }
  block_sum<3>(v, sh);
  if (threadIdx.x == 0)
    for (int j = 0; j < 3; ++j) out[3 * blockIdx.x + j] = v[j];
}

hipError_t launch_radial(int dtype, const void* pop, const uint32_t* links, int nx, int ny, int nz,
                         const double* c, int periodic, int nbins, double* P, double* shells,
                         hipStream_t s) {
  const size_t N = (size_t)nx * ny * nz;
  const int blocks = (int)((N + 255) / 256 > 8192 ? 8192 : (N + 255) / 256);
  if (dtype == 0)
    hipLaunchKernelGGL(k_radial_split<double>, dim3(blocks), dim3(256), 0, s, (const double*)pop,
                       links, nx, ny, nz, c[0], c[1], c[2], nbins, periodic, P);
  else
    hipLaunchKernelGGL(k_radial_split<float>, dim3(blocks), dim3(256), 0, s, (const float*)pop,
                       links, nx, ny, nz, c[0], c[1], c[2], nbins, periodic, P);
  hipLaunchKernelGGL(k_radial_shells, dim3(nbins), dim3(256), 0, s, P, (int)N, shells);
  return hipGetLastError();
}

hipError_t launch_pressure(int dtype, const void* pop, const uint32_t* links, int nx, int ny,
                           int nz, const PhysD& ph, void* rho, double* P, hipStream_t s) {
  hipError_t e = launch_stream_density(dtype, pop, links, rho, nx, ny, nz, s);
  if (e != hipSuccess) return e;
  const size_t N = (size_t)nx * ny * nz;
  const int blocks = (int)((N + 255) / 256 > 8192 ? 8192 : (N + 255) / 256);
  if (dtype == 0)
    hipLaunchKernelGGL(k_pressure<double>, dim3(blocks), dim3(256), 0, s, (const double*)pop, links,
                       (const double*)rho, nx, ny, nz, ph, P);
  else
    hipLaunchKernelGGL(k_pressure<float>, dim3(blocks), dim3(256), 0, s, (const float*)pop, links,
                       (const float*)rho, nx, ny, nz, phys_cast<float>(ph), P);
  return hipGetLastError();
}

hipError_t launch_plane_tension(int nx, int ny, int nz, const double* P, double* profile,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_plane_tension, dim3(nz), dim3(256), 0, s, nx, ny, nz, P, profile);
  return hipGetLastError();
}

// STREAM copy of n 8-byte words: the attainable HBM rate of a plain
// read-once write-once sweep, the reference for the step's rate.
__global__ __launch_bounds__(256) void k_stream_copy(const double* __restrict__ a,
                                                     double* __restrict__ b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// Layout ceiling: the fused step's data movement without its arithmetic.
// Every fluid node pulls its 38 populations exactly as the step does
// (periodic neighbours, bounce-back from the link mask) and stores them
// unchanged at its own index of dst; wall nodes are skipped.
template <typename real>
__global__ __launch_bounds__(256) void k_pull_copy(const real* __restrict__ src,
                                                   const uint32_t* __restrict__ links,
                                                   real* __restrict__ dst, int nx, int ny,
                                                   int nz) {
  const int N = nx * ny * nz;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    const uint32_t lb = links[i];
    if (lb & SELF_SOLID) continue;
    int xs[3], ys[3], zs[3];
    axis3(i % nx, nx, xs);
    axis3((i / nx) % ny, ny, ys);
    axis3(i / (nx * ny), nz, zs);
    real n[38];
    const PopGeo g = pop_geo(nx, ny, nz);
    pull38(src, g, xs, ys, zs, nx, lb, n);
    const size_t si = pop_slot(g, zs[1], ys[1] * nx + xs[1]);
#pragma unroll
    for (int k = 0; k < 38; ++k) dst[(k / Q) * (size_t)g.sp + si + (k % Q) * PBLK] = n[k];
  }
}

hipError_t launch_pull_copy(int dtype, const void* src, const uint32_t* links, void* dst, int nx,
                            int ny, int nz, hipStream_t s) {
  const size_t N = (size_t)nx * ny * nz;
  const unsigned g = (unsigned)((N + 255) / 256);
  if (dtype == 0)
    hipLaunchKernelGGL(k_pull_copy<double>, dim3(g), dim3(256), 0, s, (const double*)src, links,
                       (double*)dst, nx, ny, nz);
  else
    hipLaunchKernelGGL(k_pull_copy<float>, dim3(g), dim3(256), 0, s, (const float*)src, links,
                       (float*)dst, nx, ny, nz);
  return hipGetLastError();
}

hipError_t launch_stream_copy(const double* src, double* dst, size_t n, hipStream_t s) {
  const size_t g = (n + 255) / 256;
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)(g > 65536 ? 65536 : g)), dim3(256), 0, s, src,
                     dst, n);
  return hipGetLastError();
}

}  // namespace scd
