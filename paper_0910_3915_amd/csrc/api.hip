// api.hip -- host side of the libscdrop C ABI (see include/scdrop.h):
// handles, parameter validation, work-area layout, launch sequencing with
// ping-pong buffers, observables read-back, the checkpointed adjoint driver,
// HIP graph capture, the tile autotuner and the batched launch.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <iomanip>
#include <sstream>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "scdrop.h"

// A roctx range around an entry point (host side: the enqueue, or the whole
// call where it synchronises), visible in rocprofv3 --marker-trace; without
// a profiler attached a push and a pop cost a few nanoseconds.
namespace {
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};
}  // namespace

using namespace scd;

namespace {

thread_local std::string g_err;

scd_status fail(scd_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return fail(SCD_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t real_size(int dtype) { return dtype == SCD_F64 ? 8 : 4; }

// Elements of one population buffer in the blocked layout (both species).
size_t pop_elems(const scd_params* p) { return 2 * (size_t)pop_geo(p->nx, p->ny, p->nz).sp; }

struct WorkLayout {
  size_t links, partials, result, phi, ca, planes, rho, adj_partials, adj_acc, adj_dparams, q, d, e,
      jm, total;
};

WorkLayout work_layout(const scd_params* p) {
  const size_t N = (size_t)p->nx * p->ny * p->nz;
  const size_t rs = real_size(p->dtype);
  WorkLayout w{};
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
  w.links = take(N * 4);
  w.partials = take((size_t)RED_BLOCKS * RED_STRIDE * 8);
  w.result = take(16 * 8);
  w.phi = take((2 * (size_t)p->nx * p->ny + p->nz) * 8);
  w.ca = take(CA_SLOTS * 8);
  w.planes = take((size_t)p->nz * 8);  // plane means of the tension integrand
  w.rho = take(2 * N * rs);            // post-stream densities (pressure, adjoint)
  if (p->flags & SCD_WITH_ADJOINT) {
    w.adj_partials = take((size_t)ADJ_BLOCKS * RED_STRIDE * 8);
    w.adj_acc = take((size_t)ADJ_BLOCKS * RED_STRIDE * 8);  // partials summed over steps
    w.adj_dparams = take(16 * 8);  // [0, 8): last step, [8, 16): accumulator
    w.q = take(6 * N * rs);
    w.d = take(2 * N * rs);
    w.e = take(3 * N * rs);  // dL/du' / R, shared by both species
    w.jm = take(6 * N * rs);  // post-stream momenta of the state a plain reverse step reads
  }
  w.total = off;
  return w;
}

scd_status validate(const scd_params* p) {
  if (!p) return fail(SCD_EINVAL, "params is NULL");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1)
    return fail(SCD_EINVAL, "dimensions must be >= 1 (got %d %d %d)", p->nx, p->ny, p->nz);
  const double N = (double)p->nx * p->ny * p->nz;
  if (N >= (double)(1 << 30)) return fail(SCD_EINVAL, "lattice too large (%.0f nodes)", N);
  if (p->nz >= 65536) return fail(SCD_EINVAL, "nz must be < 65536");
  if (p->dtype != SCD_F64 && p->dtype != SCD_F32) return fail(SCD_EINVAL, "bad dtype %d", p->dtype);
  // 32-bit byte offsets within one species (blocked layout: planes padded to
  // whole 32-node blocks)
  const double slots = 32.0 * std::ceil((double)p->nx * p->ny / 32.0) * p->nz;
  if (19.0 * slots * (p->dtype == SCD_F64 ? 8 : 4) >= 4294967296.0)
    return fail(SCD_EUNSUPPORTED, "19 velocities of %.0f node slots exceed 4 GiB per species",
                slots);
  if (p->psi != SCD_PSI_RHO && p->psi != SCD_PSI_EXP) return fail(SCD_EINVAL, "bad psi %d", p->psi);
  for (int a = 0; a < 2; ++a) {
    if (!(p->tau[a] > 0.5) || !std::isfinite(p->tau[a]))
      return fail(SCD_EINVAL, "tau[%d] = %g must be > 1/2", a, p->tau[a]);
    if (!(p->rho_wall[a] >= 0.0) || !std::isfinite(p->rho_wall[a]))
      return fail(SCD_EINVAL, "rho_wall[%d] = %g must be >= 0", a, p->rho_wall[a]);
    if (!(p->g_wall[a] >= 0.0) || !std::isfinite(p->g_wall[a]))
      return fail(SCD_EINVAL, "g_wall[%d] = %g must be >= 0", a, p->g_wall[a]);
  }
  if (!(p->g_ab >= 0.0) || !std::isfinite(p->g_ab)) return fail(SCD_EINVAL, "g_ab = %g must be >= 0", p->g_ab);
  if (!std::isfinite(p->w_axis) || !std::isfinite(p->w_diag)) return fail(SCD_EINVAL, "bad weights");
  return SCD_OK;
}

PhysD make_phys(const scd_params* p) {
  PhysD ph;
  for (int a = 0; a < 2; ++a) {
    ph.tau[a] = p->tau[a];
    ph.inv_tau[a] = 1.0 / p->tau[a];
    ph.gw[a] = p->g_wall[a];
    ph.psiw[a] = p->psi == SCD_PSI_EXP ? 1.0 - std::exp(-p->rho_wall[a]) : p->rho_wall[a];
    ph.dpsiw[a] = p->psi == SCD_PSI_EXP ? std::exp(-p->rho_wall[a]) : 1.0;
  }
  ph.gab = p->g_ab;
  ph.wa = p->w_axis;
  ph.wd = p->w_diag;
  ph.psi_form = p->psi;
  return ph;
}

}  // namespace

struct scd_lattice {
  scd_params p;
  PhysD ph;
  size_t N;
  WorkLayout wl;
  const uint8_t* solid;
  void* pop[2];
  int cur;
  char* work;
  hipStream_t stream;
  int64_t step;
  int variant, zc, remap;
  hipGraph_t graph;
  hipGraphExec_t gexec;
  int64_t graph_steps;
  int graph_cur;
  bool batch_view;  // buffers belong to a batch
  int64_t ckpt_base;  // step at which the last checkpointed forward began
  void* mom_cache = nullptr;      // caller buffer of moment fields of recomputed steps
  int64_t mom_cache_steps = 0;    // ... and how many steps (8 x N reals each) it holds
  // mass-drift watchdog: tolerance (0: off), reference masses (taken by the
  // first scd_observables after the state was set) and the last drift
  double watch_tol = 0.0;
  bool mass_ref_ok = false;
  double mass_ref[2] = {0.0, 0.0};
  double drift[2] = {0.0, 0.0};
  uint32_t* links() const { return (uint32_t*)(work + wl.links); }
  double* wd(size_t off) const { return (double*)(work + off); }
  void* wv(size_t off) const { return (void*)(work + off); }
};

namespace {

// Defaults from variant sweeps on MI355X (128 x 128 x 64 and larger
// droplets): FP64 marches three planes per barrier on 32 x 4 tiles at one
// wave per SIMD (its registers do not fit two), FP32 two planes per barrier
// on 64 x 4 tiles at two waves per SIMD.
int default_variant(int dtype) {
  int v = dtype == SCD_F64 ? variant_find(32, 4, 7, 1) : variant_find(64, 4, 6, 2);
  return v < 0 ? 0 : v;
}

int device_cus() {
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return cus > 0 ? cus : 256;
}

// z-chunk from a wave-count model: each tile column is cut into chunks of zc
// planes, a chunk reads zc + 2 planes, and the chunks run in rounds of one
// workgroup per compute unit, so a step costs about rounds * (zc + 2) plane
// times.  Every chunk count per column is tried with its shortest chunk
// length (at least 4 planes); among those that give every compute unit a
// workgroup the cheapest wins (the shorter chunk on a tie).  A lattice too
// small to fill the chip takes 4-plane chunks.
int default_zc(const scd_params& p, int variant) {
  int tx, ty, var, wpe;
  variant_at(variant, &tx, &ty, &var, &wpe);
  const long cols = (long)((p.nx + tx - 1) / tx) * ((p.ny + ty - 1) / ty);
  const long cus = device_cus();
  int best = std::min(4, p.nz);
  long best_cost = -1;
  for (int nch = (p.nz + 3) / 4; nch >= 1; --nch) {
    const int zc = (p.nz + nch - 1) / nch;
    const long blocks = cols * ((p.nz + zc - 1) / zc);
    if (blocks < cus) continue;
    const long cost = (blocks + cus - 1) / cus * (zc + 2);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = zc;
    }
  }
  return best;
}

void default_tile(scd_lattice* h) {
  h->variant = default_variant(h->p.dtype);
  h->zc = default_zc(h->p, h->variant);
  h->remap = 1;
  // Boxes that give every CU a tile-column chunk of at least 8 planes on
  // the taller tile: the two-rows-per-thread march, 64 x 8 in FP32 and
  // 32 x 8 in FP64 (0.29 and 0.33 halo nodes per interior node against
  // 0.55 and 0.59 on 64 x 4 and 32 x 4).  Measured on 128 x 128 x 64:
  // FP32 75.5 against 81.3 us per step, FP64 141.6 against 142.2; on
  // 256 x 256 x 128 at 64-plane chunks: 555.7 against 635.7 and 1161
  // against 1290.
  const bool f32 = h->p.dtype == SCD_F32;
  const int v = f32 ? variant_find(64, 8, 9, 2) : variant_find(32, 8, 9, 1);
  const int tx = f32 ? 64 : 32;
  const long cols = (long)((h->p.nx + tx - 1) / tx) * ((h->p.ny + 7) / 8);
  if (v >= 0 && cols * (h->p.nz / 8) >= device_cus()) {
    h->variant = v;
    h->zc = default_zc(h->p, v);
  }
}

scd_status enqueue_steps(scd_lattice* h, int64_t nsteps) {
  for (int64_t s = 0; s < nsteps; ++s) {
    HIPCHK(launch_step(h->p.dtype, h->pop[h->cur], h->pop[1 - h->cur], h->links(), h->p.nx, h->p.ny,
                       h->p.nz, h->ph, h->variant, h->zc, h->remap, h->stream));
    h->cur ^= 1;
    h->step += 1;
  }
  return SCD_OK;
}

void drop_graph(scd_lattice* h) {
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->gexec = nullptr;
  h->graph = nullptr;
  h->graph_steps = 0;
}

scd_status check_cfg(const scd_lattice* h, const scd_ca_cfg* c) {
  if (!c) return fail(SCD_EINVAL, "ca cfg is NULL");
  if (c->ic < 0 || c->ic >= h->p.nx || c->jc < 0 || c->jc >= h->p.ny)
    return fail(SCD_EINVAL, "column (%d, %d) outside the lattice", c->ic, c->jc);
  if (c->z_solid_top < 0 || c->offset < 1 || c->z_solid_top + c->offset >= h->p.nz - 1)
    return fail(SCD_EINVAL, "reference layer %d + %d outside the lattice", c->z_solid_top, c->offset);
  if (!(c->eps > 0.0)) return fail(SCD_EINVAL, "eps must be > 0");
  return SCD_OK;
}

CaDev ca_dev(const scd_ca_cfg* c) { return CaDev{c->ic, c->jc, c->z_solid_top, c->offset, c->eps}; }

scd_status read_ca(scd_lattice* h, scd_ca* out, double* status_out,
                   const double* d_slots = nullptr) {
  double r[CA_SLOTS];
  HIPCHK(hipMemcpyAsync(r, d_slots ? d_slots : h->wd(h->wl.ca), sizeof(r), hipMemcpyDeviceToHost,
                        h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (out) {
    out->theta_e1 = r[0]; out->h_e1 = r[1]; out->a_e1 = r[2]; out->R_e1 = r[3];
    out->aref_e1 = r[4]; out->H_e1 = r[5];
    out->theta_e2 = r[6]; out->h_e2 = r[7]; out->a_e2 = r[8]; out->R_e2 = r[9];
    out->aref_e2 = r[10]; out->H_e2 = r[11];
    out->cx = r[12]; out->cy = r[13];
    out->flags = (int32_t)r[14];
    out->pad = 0;
  }
  if (status_out) *status_out = r[15];
  return SCD_OK;
}

}  // namespace

extern "C" {

scd_status scd_stream_copy(const void* d_src, void* d_dst, size_t bytes, void* stream) {
  if (!d_src || !d_dst) return fail(SCD_EINVAL, "NULL pointer");
  if (bytes % 8 || ((uintptr_t)d_src | (uintptr_t)d_dst) % 8)
    return fail(SCD_EINVAL, "size and pointers must be multiples of 8 bytes");
  const uintptr_t a = (uintptr_t)d_src, b = (uintptr_t)d_dst;
  if (a < b + bytes && b < a + bytes) return fail(SCD_EINVAL, "source and destination overlap");
  if (bytes == 0) return SCD_OK;
  HIPCHK(launch_stream_copy((const double*)d_src, (double*)d_dst, bytes / 8,
                            (hipStream_t)stream));
  return SCD_OK;
}

const char* scd_last_error(void) { return g_err.c_str(); }
const char* scd_version(void) { return "scdrop 1.0 (gfx950)"; }

scd_status scd_sizes(const scd_params* p, size_t* pop_bytes, size_t* work_bytes) {
  scd_status st = validate(p);
  if (st) return st;
  if (pop_bytes) *pop_bytes = pop_elems(p) * real_size(p->dtype);
  if (work_bytes) *work_bytes = work_layout(p).total;
  return SCD_OK;
}

scd_status scd_create(const scd_params* p, const uint8_t* d_solid, void* d_pop0, void* d_pop1,
                      void* d_work, void* stream, scd_lattice** out) {
  scd_status st = validate(p);
  if (st) return st;
  if (!out || !d_solid || !d_pop0 || !d_pop1 || !d_work)
    return fail(SCD_EINVAL, "NULL buffer passed to scd_create");
  if (d_pop0 == d_pop1) return fail(SCD_EINVAL, "the two population buffers must differ");
  if (((uintptr_t)d_pop0 | (uintptr_t)d_pop1 | (uintptr_t)d_work) & 255)
    return fail(SCD_EINVAL, "device buffers must be 256-byte aligned");
  scd_lattice* h = new scd_lattice();
  h->p = *p;
  h->ph = make_phys(p);
  h->N = (size_t)p->nx * p->ny * p->nz;
  h->wl = work_layout(p);
  h->solid = d_solid;
  h->pop[0] = d_pop0;
  h->pop[1] = d_pop1;
  h->cur = 0;
  h->work = (char*)d_work;
  h->stream = (hipStream_t)stream;
  h->step = 0;
  h->graph = nullptr;
  h->gexec = nullptr;
  h->graph_steps = 0;
  h->graph_cur = 0;
  h->batch_view = false;
  h->ckpt_base = 0;
  default_tile(h);
  hipError_t e = launch_links(d_solid, h->links(), p->nx, p->ny, p->nz, h->stream);
  if (e != hipSuccess) {
    delete h;
    return fail(SCD_EDEVICE, "link-mask kernel: %s", hipGetErrorString(e));
  }
  *out = h;
  return SCD_OK;
}

scd_status scd_destroy(scd_lattice* h) {
  if (!h) return SCD_OK;
  drop_graph(h);
  delete h;
  return SCD_OK;
}

scd_status scd_set_params(scd_lattice* h, const scd_params* p) {
  if (!h) return fail(SCD_EINVAL, "NULL handle");
  scd_status st = validate(p);
  if (st) return st;
  if (p->nx != h->p.nx || p->ny != h->p.ny || p->nz != h->p.nz || p->dtype != h->p.dtype ||
      p->flags != h->p.flags)
    return fail(SCD_EINVAL, "dims, dtype and flags are fixed at creation");
  h->p = *p;
  h->ph = make_phys(p);
  drop_graph(h);  // captured kernels carry the old parameters
  return SCD_OK;
}

scd_status scd_set_stream(scd_lattice* h, void* stream) {
  if (!h) return fail(SCD_EINVAL, "NULL handle");
  h->stream = (hipStream_t)stream;
  drop_graph(h);
  return SCD_OK;
}

scd_status scd_init_equilibrium(scd_lattice* h, const double* d_rho_a, const double* d_rho_b) {
  if (!h || !d_rho_a || !d_rho_b) return fail(SCD_EINVAL, "NULL argument");
  // the other buffer's wall-node entries are never written by a step: zero
  // it so that every state copy is fully defined
  HIPCHK(launch_fill(h->p.dtype, h->pop[1 - h->cur], pop_elems(&h->p), 0.0, h->stream));
  HIPCHK(launch_init(h->p.dtype, h->pop[h->cur], d_rho_a, d_rho_b, h->links(), h->p.nx, h->p.ny,
                     h->p.nz, h->stream));
  h->step = 0;
  h->mass_ref_ok = false;
  return SCD_OK;
}

scd_status scd_step(scd_lattice* h, int64_t nsteps) {
  TraceRange trace_("scd_step");
  if (!h) return fail(SCD_EINVAL, "NULL handle");
  if (nsteps < 0) return fail(SCD_EINVAL, "nsteps < 0");
  return enqueue_steps(h, nsteps);
}

int64_t scd_step_count(const scd_lattice* h) { return h ? h->step : -1; }

scd_status scd_get_state(scd_lattice* h, void* d_dst) {
  if (!h || !d_dst) return fail(SCD_EINVAL, "NULL argument");
  HIPCHK(hipMemcpyAsync(d_dst, h->pop[h->cur], pop_elems(&h->p) * real_size(h->p.dtype),
                        hipMemcpyDeviceToDevice, h->stream));
  return SCD_OK;
}

scd_status scd_set_state(scd_lattice* h, const void* d_src, int64_t step) {
  if (!h || !d_src) return fail(SCD_EINVAL, "NULL argument");
  HIPCHK(hipMemcpyAsync(h->pop[h->cur], d_src, pop_elems(&h->p) * real_size(h->p.dtype),
                        hipMemcpyDeviceToDevice, h->stream));
  h->step = step;
  h->mass_ref_ok = false;
  return SCD_OK;
}

// Repacking between the plain and the blocked population layouts.
static scd_status pop_repack(const scd_lattice* h, const void* src, void* dst, bool to_blocked) {
  if (!h || !src || !dst) return fail(SCD_EINVAL, "NULL argument");
  const size_t rs = real_size(h->p.dtype);
  const size_t plain = 2 * Q * h->N * rs, blocked = pop_elems(&h->p) * rs;
  const uintptr_t s0 = (uintptr_t)src, d0 = (uintptr_t)dst;
  const size_t sn = to_blocked ? plain : blocked, dn = to_blocked ? blocked : plain;
  if (s0 < d0 + dn && d0 < s0 + sn) return fail(SCD_EINVAL, "source and destination overlap");
  if ((s0 | d0) % rs) return fail(SCD_EINVAL, "buffers must be aligned to the element size");
  HIPCHK(launch_pop_repack(h->p.dtype, src, dst, h->p.nx, h->p.ny, h->p.nz, to_blocked, h->stream));
  return SCD_OK;
}

scd_status scd_pop_pack(const scd_lattice* h, const void* d_plain, void* d_blocked) {
  return pop_repack(h, d_plain, d_blocked, true);
}

scd_status scd_pop_unpack(const scd_lattice* h, const void* d_blocked, void* d_plain) {
  return pop_repack(h, d_blocked, d_plain, false);
}

scd_status scd_fill_state(scd_lattice* h, double value) {
  if (!h) return fail(SCD_EINVAL, "NULL handle");
  HIPCHK(launch_fill(h->p.dtype, h->pop[h->cur], pop_elems(&h->p), value, h->stream));
  h->mass_ref_ok = false;
  return SCD_OK;
}

scd_status scd_pull_copy(scd_lattice* h) {
  if (!h) return fail(SCD_EINVAL, "NULL handle");
  HIPCHK(launch_pull_copy(h->p.dtype, h->pop[h->cur], h->links(), h->pop[1 - h->cur], h->p.nx,
                          h->p.ny, h->p.nz, h->stream));
  return SCD_OK;
}

scd_status scd_pressure_tensor(scd_lattice* h, double* d_P) {
  TraceRange trace_("scd_pressure_tensor");
  if (!h || !d_P) return fail(SCD_EINVAL, "NULL argument");
  HIPCHK(launch_pressure(h->p.dtype, h->pop[h->cur], h->links(), h->p.nx, h->p.ny, h->p.nz, h->ph,
                         h->wd(h->wl.rho), d_P, h->stream));
  return SCD_OK;
}

scd_status scd_surface_tension_z(scd_lattice* h, double* d_P, double* h_gamma,
                                 double* h_profile) {
  TraceRange trace_("scd_surface_tension_z");
  if (!h || !d_P || !h_gamma) return fail(SCD_EINVAL, "NULL argument");
  scd_status st = scd_pressure_tensor(h, d_P);
  if (st) return st;
  double* planes = (double*)h->wd(h->wl.planes);
  HIPCHK(launch_plane_tension(h->p.nx, h->p.ny, h->p.nz, d_P, planes, h->stream));
  std::vector<double> prof(h->p.nz);
  HIPCHK(hipMemcpyAsync(prof.data(), planes, prof.size() * 8, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  double total = 0.0;  // planes summed in order z = 0, 1, ...
  for (int z = 0; z < h->p.nz; ++z) total += prof[z];
  *h_gamma = total;
  if (h_profile) std::copy(prof.begin(), prof.end(), h_profile);
  return SCD_OK;
}

scd_status scd_radial_tension(scd_lattice* h, double* d_P, const double* h_center, double rmax,
                              int32_t nbins, double* h_profile, double* h_phi_profile,
                              double* h_Rs, double* h_gamma) {
  return scd_radial_tension_axes(h, d_P, h_center, 7, rmax, nbins, h_profile, h_phi_profile, h_Rs,
                                 h_gamma);
}

scd_status scd_radial_tension_axes(scd_lattice* h, double* d_P, const double* h_center,
                                   int32_t periodic, double rmax, int32_t nbins,
                                   double* h_profile, double* h_phi_profile, double* h_Rs,
                                   double* h_gamma) {
  TraceRange trace_("scd_radial_tension_axes");
  if (!h || !d_P || !h_center || !h_Rs || !h_gamma) return fail(SCD_EINVAL, "NULL argument");
  if (periodic < 0 || periodic > 7) return fail(SCD_EINVAL, "periodic mask must be in [0, 7]");
  const int maxb = RED_BLOCKS * RED_STRIDE / 3;
  if (nbins < 2 || nbins > maxb) return fail(SCD_EINVAL, "nbins must be in [2, %d]", maxb);
  scd_status st = scd_pressure_tensor(h, d_P);
  if (st) return st;
  double* shells = (double*)h->wd(h->wl.partials);
  HIPCHK(launch_radial(h->p.dtype, h->pop[h->cur], h->links(), h->p.nx, h->p.ny, h->p.nz,
                       h_center, periodic, nbins, d_P, shells, h->stream));
  std::vector<double> sh(3 * (size_t)nbins);
  HIPCHK(hipMemcpyAsync(sh.data(), shells, sh.size() * 8, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  std::vector<double> prof(nbins), phi(nbins);
  for (int b = 0; b < nbins; ++b) {
    const double n = sh[3 * b + 2];
    prof[b] = n > 0 ? sh[3 * b] / n : 0.0;
    phi[b] = n > 0 ? sh[3 * b + 1] / n : 0.0;
  }
  if (h_profile) std::copy(prof.begin(), prof.end(), h_profile);
  if (h_phi_profile) std::copy(phi.begin(), phi.end(), h_phi_profile);
  double R = NAN;
  for (int b = 0; b + 1 < nbins; ++b)
    if (phi[b] > 0.0 && phi[b + 1] <= 0.0) {
      R = (b + 0.5) + phi[b] / (phi[b] - phi[b + 1]);
      break;
    }
  *h_Rs = R;
  if (std::isnan(R)) {
    *h_gamma = NAN;
    return fail(SCD_ENOINTERFACE, "phi has no outward crossing about the centre");
  }
  double g = 0.0;
  for (int b = 0; b < nbins && b + 0.5 <= rmax; ++b) {
    const double rb = b + 0.5;
    g += (rb / R) * (rb / R) * prof[b];
  }
  *h_gamma = g;
  return SCD_OK;
}

double scd_young_angle(double gamma_sg, double gamma_sl, double gamma_lg) {
  const double c = std::min(1.0, std::max(-1.0, (gamma_sg - gamma_sl) / gamma_lg));
  return std::acos(c) * (180.0 / M_PI);
}

double scd_huang_angle(const scd_params* p, double rho_in, double rho_out) {
  if (!p) return NAN;
  auto psi = [&](double r) { return p->psi == SCD_PSI_EXP ? 1.0 - std::exp(-r) : r; };
  const double ads_a = p->g_wall[0] * psi(p->rho_wall[1]);  // repulsion felt by A
  const double ads_b = p->g_wall[1] * psi(p->rho_wall[0]);  // ... by B
  return scd_young_angle(ads_b, ads_a, p->g_ab * (rho_in - rho_out) / 2.0);
}

scd_status scd_density(scd_lattice* h, double* d_rho) {
  if (!h || !d_rho) return fail(SCD_EINVAL, "NULL argument");
  HIPCHK(launch_density(h->p.dtype, h->pop[h->cur], h->links(), d_rho, h->p.nx, h->p.ny, h->p.nz,
                        h->stream));
  return SCD_OK;
}

scd_status scd_observables(scd_lattice* h, scd_obs* out) {
  TraceRange trace_("scd_observables");
  if (!h || !out) return fail(SCD_EINVAL, "NULL argument");
  HIPCHK(launch_observables(h->p.dtype, h->pop[h->cur], h->links(), h->p.nx, h->p.ny, h->p.nz,
                            h->wd(h->wl.partials), h->wd(h->wl.result), h->stream));
  double r[6];
  HIPCHK(hipMemcpyAsync(r, h->wd(h->wl.result), sizeof(r), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  out->mass[0] = r[0];
  out->mass[1] = r[1];
  out->momentum[0] = r[2];
  out->momentum[1] = r[3];
  out->momentum[2] = r[4];
  out->finite = r[5] == 0.0 ? 1 : 0;
  out->pad = 0;
  out->step = h->step;
  if (!out->finite) return fail(SCD_ENONFINITE, "%.0f non-finite populations", r[5]);
  // the watchdog: relative change of each species' mass since the reference
  if (!h->mass_ref_ok) {
    h->mass_ref[0] = r[0];
    h->mass_ref[1] = r[1];
    h->mass_ref_ok = true;
  }
  for (int a = 0; a < 2; ++a)
    h->drift[a] = h->mass_ref[a] != 0.0 ? (r[a] - h->mass_ref[a]) / h->mass_ref[a] : r[a];
  const double worst = std::max(std::fabs(h->drift[0]), std::fabs(h->drift[1]));
  if (h->watch_tol > 0.0 && worst > h->watch_tol)
    return fail(SCD_EDRIFT, "mass drift %.3e exceeds the watchdog tolerance %.3e at step %lld", worst,
                h->watch_tol, (long long)h->step);
  return SCD_OK;
}

scd_status scd_set_mass_watchdog(scd_lattice* h, double rel_tol) {
  if (!h) return fail(SCD_EINVAL, "NULL handle");
  if (!(rel_tol >= 0.0)) return fail(SCD_EINVAL, "watchdog tolerance must be >= 0");
  h->watch_tol = rel_tol;
  return SCD_OK;
}

scd_status scd_mass_drift(const scd_lattice* h, double* h_drift) {
  if (!h || !h_drift) return fail(SCD_EINVAL, "NULL argument");
  h_drift[0] = h->drift[0];
  h_drift[1] = h->drift[1];
  return SCD_OK;
}

scd_status scd_contact_angle(scd_lattice* h, const scd_ca_cfg* cfg, scd_ca* out) {
  TraceRange trace_("scd_contact_angle");
  if (!h || !out) return fail(SCD_EINVAL, "NULL argument");
  scd_status st = check_cfg(h, cfg);
  if (st) return st;
  HIPCHK(launch_contact_angle(h->p.dtype, h->pop[h->cur], h->links(), h->p.nx, h->p.ny, h->p.nz,
                              ca_dev(cfg), h->wd(h->wl.phi), h->wd(h->wl.partials),
                              h->wd(h->wl.ca), h->stream));
  double status;
  st = read_ca(h, out, &status);
  if (st) return st;
  if (status != 0.0) return fail(SCD_ENOINTERFACE, "no droplet on column (%d, %d)", cfg->ic, cfg->jc);
  return SCD_OK;
}

scd_status scd_contact_angle_static(scd_lattice* h, const scd_ca_cfg* cfg, scd_ca* out) {
  TraceRange trace_("scd_contact_angle_static");
  if (!h || !out) return fail(SCD_EINVAL, "NULL argument");
  scd_status st = check_cfg(h, cfg);
  if (st) return st;
  if ((size_t)h->p.nx * h->p.ny > CA_STATIC_MAX_PLANE || (size_t)h->p.nz > CA_STATIC_MAX_NZ)
    return fail(SCD_EUNSUPPORTED,
                "static contact-angle scratch holds planes of at most %zu nodes and %zu planes "
                "(lattice %d x %d x %d); use scd_contact_angle",
                CA_STATIC_MAX_PLANE, CA_STATIC_MAX_NZ, h->p.nx, h->p.ny, h->p.nz);
  double *phi, *part, *res;
  HIPCHK(ca_static_scratch(&phi, &part, &res));
  HIPCHK(launch_contact_angle(h->p.dtype, h->pop[h->cur], h->links(), h->p.nx, h->p.ny, h->p.nz,
                              ca_dev(cfg), phi, part, res, h->stream));
  double status;
  st = read_ca(h, out, &status, res);
  if (st) return st;
  if (status != 0.0) return fail(SCD_ENOINTERFACE, "no droplet on column (%d, %d)", cfg->ic, cfg->jc);
  return SCD_OK;
}

scd_status scd_ca_seed(scd_lattice* h, const scd_ca_cfg* cfg, double dL_dtheta, void* d_lambda) {
  if (!h || !d_lambda) return fail(SCD_EINVAL, "NULL argument");
  scd_status st = check_cfg(h, cfg);
  if (st) return st;
  HIPCHK(launch_contact_angle(h->p.dtype, h->pop[h->cur], h->links(), h->p.nx, h->p.ny, h->p.nz,
                              ca_dev(cfg), h->wd(h->wl.phi), h->wd(h->wl.partials),
                              h->wd(h->wl.ca), h->stream));
  HIPCHK(launch_ca_seed(h->p.dtype, h->links(), h->p.nx, h->p.ny, h->p.nz, ca_dev(cfg),
                        h->wd(h->wl.phi), h->wd(h->wl.ca), dL_dtheta, d_lambda, h->stream));
  scd_ca ca;
  double status;
  st = read_ca(h, &ca, &status);
  if (st) return st;
  if (status != 0.0 || (ca.flags & SCD_CA_E2_EMPTY))
    return fail(SCD_ENOINTERFACE, "no droplet for the E2 seed");
  return SCD_OK;
}

static scd_status adjoint_enqueue(scd_lattice* h, const void* state_t, const void* lam_in,
                                  void* lam_out, bool accumulate,
                                  const void* mom_cached = nullptr) {
  HIPCHK(launch_adjoint(h->p.dtype, state_t, lam_in, lam_out, h->links(), h->p.nx, h->p.ny,
                        h->p.nz, h->ph, h->wv(h->wl.rho), h->wv(h->wl.jm), mom_cached, h->wv(h->wl.q),
                        h->wv(h->wl.d), h->wv(h->wl.e), h->wd(h->wl.adj_partials),
                        h->wd(h->wl.adj_dparams),
                        accumulate ? h->wd(h->wl.adj_acc) : nullptr, h->stream));
  return SCD_OK;
}

scd_status scd_adjoint_reset(scd_lattice* h) {
  if (!h) return fail(SCD_EINVAL, "NULL handle");
  if (!(h->p.flags & SCD_WITH_ADJOINT))
    return fail(SCD_EUNSUPPORTED, "lattice created without SCD_WITH_ADJOINT");
  HIPCHK(launch_zero(h->wd(h->wl.adj_acc), ADJ_BLOCKS * RED_STRIDE, h->stream));
  return SCD_OK;
}

scd_status scd_adjoint_read(scd_lattice* h, double* h_acc) {
  if (!h || !h_acc) return fail(SCD_EINVAL, "NULL argument");
  if (!(h->p.flags & SCD_WITH_ADJOINT))
    return fail(SCD_EUNSUPPORTED, "lattice created without SCD_WITH_ADJOINT");
  HIPCHK(launch_adjoint_sum(h->p.dtype, h->wd(h->wl.adj_acc), h->N, h->wd(h->wl.adj_dparams) + 8,
                            h->stream));
  HIPCHK(hipMemcpyAsync(h_acc, h->wd(h->wl.adj_dparams) + 8, 5 * sizeof(double),
                        hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return SCD_OK;
}

scd_status scd_adjoint_step(scd_lattice* h, const void* d_state_t, const void* d_lam_in,
                            void* d_lam_out, double* h_dparams) {
  TraceRange trace_("scd_adjoint_step");
  if (!h || !d_state_t || !d_lam_in || !d_lam_out) return fail(SCD_EINVAL, "NULL argument");
  if (!(h->p.flags & SCD_WITH_ADJOINT))
    return fail(SCD_EUNSUPPORTED, "lattice created without SCD_WITH_ADJOINT");
  if (d_lam_in == d_lam_out) return fail(SCD_EINVAL, "lambda in and out must not alias");
  scd_status st = adjoint_enqueue(h, d_state_t, d_lam_in, d_lam_out, h_dparams == nullptr);
  if (st) return st;
  if (!h_dparams) return SCD_OK;  // accumulated on the device, no synchronisation
  double g[5];
  HIPCHK(hipMemcpyAsync(g, h->wv(h->wl.adj_dparams), sizeof(g), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  for (int j = 0; j < 5; ++j) h_dparams[j] += g[j];
  return SCD_OK;
}

static const double kRad2Deg = 57.295779513082320876798154814105;

scd_status scd_ckpt_forward(scd_lattice* h, const double* d_rho_a, const double* d_rho_b,
                            int64_t nsteps, int64_t K, void* d_ckpt, const scd_ca_cfg* cfg,
                            double target_deg, double* h_out) {
  TraceRange trace_("scd_ckpt_forward");
  if (!h || !d_ckpt || !h_out) return fail(SCD_EINVAL, "NULL argument");
  if (nsteps < 1 || K < 1) return fail(SCD_EINVAL, "nsteps and ckpt_every must be >= 1");
  if ((d_rho_a == nullptr) != (d_rho_b == nullptr))
    return fail(SCD_EINVAL, "give both densities or neither");
  scd_status st = check_cfg(h, cfg);
  if (st) return st;
  if (d_rho_a) {
    st = scd_init_equilibrium(h, d_rho_a, d_rho_b);
    if (st) return st;
  }
  h->ckpt_base = h->step;
  const size_t bytes = pop_elems(&h->p) * real_size(h->p.dtype);
  for (int64_t t = 0; t < nsteps; t += K) {
    HIPCHK(hipMemcpyAsync((char*)d_ckpt + (size_t)(t / K) * bytes, h->pop[h->cur], bytes,
                          hipMemcpyDeviceToDevice, h->stream));
    st = enqueue_steps(h, std::min(K, nsteps - t));
    if (st) return st;
  }
  scd_ca ca;
  st = scd_contact_angle(h, cfg, &ca);
  if (st) return st;
  h_out[0] = (ca.theta_e2 - target_deg) * (ca.theta_e2 - target_deg);
  h_out[1] = ca.theta_e2;
  return SCD_OK;
}

// Reverse sweep over steps [t0, t1) (relative to the checkpointed forward)
// whose starting state is in d_start: recompute the states into d_seg and
// run the adjoint steps backwards, lambda ping-ponging in lam[2].
// Recompute the states t0 .. t1 - 1 of one segment from d_start (the state
// at t0) and apply the adjoint steps t1 - 1 .. t0.  Each recomputed step
// writes its successor's slot of d_seg directly (slot j holds state
// t0 + 1 + j), so the segment costs t1 - t0 - 1 steps and no state copies.
// With a moment cache of at least t1 - t0 - 1 steps (and a step variant
// that writes moments), each recomputed step also stores the densities and
// momenta of the post-stream populations of the state it reads, and the
// adjoint of that state reads them instead of pulling its populations to
// form them; for the last state of the segment, which no recomputed step
// reads, the adjoint forms them itself.  The adjoint of a state whose
// moments are cached reads nothing else of the state, so with the cache the
// recomputed states only alternate between two slots of d_seg (state
// t0 + 1 + j in slot j mod 2): a segment then needs two states of room
// instead of t1 - t0 - 1, and long segments fit where their states would
// not.
static scd_status reverse_segment(scd_lattice* h, int64_t t0, int64_t t1, const void* d_start,
                                  void* d_seg, void* lam[2], int* lc) {
  const size_t bytes = pop_elems(&h->p) * real_size(h->p.dtype);
  const size_t mbytes = 8 * h->N * real_size(h->p.dtype);
  const bool cache = h->mom_cache && h->mom_cache_steps >= t1 - t0 - 1 &&
                     variant_writes_moments(h->variant);
  auto state = [&](int64_t t) -> const void* {
    if (t == t0) return d_start;
    const int64_t j = t - t0 - 1;
    return (const char*)d_seg + (size_t)(cache ? (j & 1) : j) * bytes;
  };
  auto mom = [&](int64_t t) -> void* {
    return cache && t + 1 < t1 ? (char*)h->mom_cache + (size_t)(t - t0) * mbytes : nullptr;
  };
  for (int64_t t = t0; t + 1 < t1; ++t)
    HIPCHK(launch_step(h->p.dtype, state(t), const_cast<void*>(state(t + 1)), h->links(), h->p.nx,
                       h->p.ny, h->p.nz, h->ph, h->variant, h->zc, h->remap, h->stream, mom(t)));
  for (int64_t t = t1 - 1; t >= t0; --t) {
    scd_status st = adjoint_enqueue(h, state(t), lam[*lc], lam[1 - *lc], true, mom(t));
    if (st) return st;
    *lc = 1 - *lc;
  }
  return SCD_OK;
}

scd_status scd_ckpt_seg_states(const scd_lattice* h, int64_t seg_len, int64_t* h_states) {
  if (!h || !h_states) return fail(SCD_EINVAL, "NULL argument");
  if (seg_len < 1) return fail(SCD_EINVAL, "segment length must be >= 1");
  const bool cache = h->mom_cache && h->mom_cache_steps >= seg_len - 1 &&
                     variant_writes_moments(h->variant);
  *h_states = cache ? std::min<int64_t>(2, seg_len - 1) : seg_len - 1;
  return SCD_OK;
}

scd_status scd_ckpt_moment_cache(scd_lattice* h, void* d_buf, int64_t nsteps) {
  if (!h) return fail(SCD_EINVAL, "NULL handle");
  if (nsteps < 0 || (nsteps > 0 && !d_buf)) return fail(SCD_EINVAL, "bad moment cache");
  h->mom_cache = nsteps > 0 ? d_buf : nullptr;
  h->mom_cache_steps = nsteps;
  return SCD_OK;
}

// After a backward sweep the lattice holds the first checkpoint (step
// ckpt_base), the start of the segment reversed last.
static scd_status backward_finish(scd_lattice* h, const void* d_ckpt, double* h_grad) {
  const size_t bytes = pop_elems(&h->p) * real_size(h->p.dtype);
  HIPCHK(hipMemcpyAsync(h->pop[h->cur], d_ckpt, bytes, hipMemcpyDeviceToDevice, h->stream));
  h->step = h->ckpt_base;
  return scd_adjoint_read(h, h_grad);
}

static scd_status backward_start(scd_lattice* h, int64_t nsteps, int64_t K, const void* d_ckpt,
                                 void* d_lam, const scd_ca_cfg* cfg, double target_deg,
                                 void* lam[2]) {
  if (!(h->p.flags & SCD_WITH_ADJOINT))
    return fail(SCD_EUNSUPPORTED, "lattice created without SCD_WITH_ADJOINT");
  if (nsteps < 1 || K < 1) return fail(SCD_EINVAL, "nsteps and checkpoint spacing must be >= 1");
  if (h->step != h->ckpt_base + nsteps)
    return fail(SCD_EINVAL, "state is at step %lld, expected %lld", (long long)h->step,
                (long long)(h->ckpt_base + nsteps));
  if (!d_ckpt || !d_lam) return fail(SCD_EINVAL, "NULL argument");
  scd_status st = check_cfg(h, cfg);
  if (st) return st;
  const size_t bytes = pop_elems(&h->p) * real_size(h->p.dtype);
  scd_ca ca;
  st = scd_contact_angle(h, cfg, &ca);
  if (st) return st;
  const double dL_dtheta = 2.0 * (ca.theta_e2 - target_deg) * kRad2Deg;  // per radian
  lam[0] = d_lam;
  lam[1] = (char*)d_lam + bytes;
  st = scd_ca_seed(h, cfg, dL_dtheta, lam[0]);
  if (st) return st;
  return scd_adjoint_reset(h);
}

scd_status scd_ckpt_backward(scd_lattice* h, int64_t nsteps, int64_t K, const void* d_ckpt,
                             void* d_seg, void* d_lam, const scd_ca_cfg* cfg, double target_deg,
                             double* h_grad) {
  TraceRange trace_("scd_ckpt_backward");
  if (!h || !d_seg || !h_grad) return fail(SCD_EINVAL, "NULL argument");
  void* lam[2];
  scd_status st = backward_start(h, nsteps, K, d_ckpt, d_lam, cfg, target_deg, lam);
  if (st) return st;
  const size_t bytes = pop_elems(&h->p) * real_size(h->p.dtype);
  int lc = 0;
  const int64_t nseg = (nsteps + K - 1) / K;
  for (int64_t s = nseg - 1; s >= 0; --s) {
    st = reverse_segment(h, s * K, std::min(nsteps, s * K + K), (const char*)d_ckpt + (size_t)s * bytes,
                         d_seg, lam, &lc);
    if (st) return st;
  }
  return backward_finish(h, d_ckpt, h_grad);
}

scd_status scd_ckpt_backward2(scd_lattice* h, int64_t nsteps, int64_t K1, int64_t K2,
                              const void* d_ckpt, void* d_mid, void* d_seg, void* d_lam,
                              const scd_ca_cfg* cfg, double target_deg, double* h_grad) {
  TraceRange trace_("scd_ckpt_backward2");
  if (!h || !d_mid || !d_seg || !h_grad) return fail(SCD_EINVAL, "NULL argument");
  if (K2 < 1 || K2 > K1) return fail(SCD_EINVAL, "need 1 <= K2 <= K1");
  void* lam[2];
  scd_status st = backward_start(h, nsteps, K1, d_ckpt, d_lam, cfg, target_deg, lam);
  if (st) return st;
  const size_t bytes = pop_elems(&h->p) * real_size(h->p.dtype);
  int lc = 0;
  const int64_t nseg = (nsteps + K1 - 1) / K1;
  for (int64_t s = nseg - 1; s >= 0; --s) {
    const int64_t t0 = s * K1, t1 = std::min(nsteps, t0 + K1);
    // level 2: checkpoints every K2 steps inside the segment
    HIPCHK(hipMemcpyAsync(h->pop[h->cur], (const char*)d_ckpt + (size_t)s * bytes, bytes,
                          hipMemcpyDeviceToDevice, h->stream));
    h->step = h->ckpt_base + t0;
    for (int64_t t = t0; t < t1; t += K2) {
      HIPCHK(hipMemcpyAsync((char*)d_mid + (size_t)((t - t0) / K2) * bytes, h->pop[h->cur], bytes,
                            hipMemcpyDeviceToDevice, h->stream));
      st = enqueue_steps(h, std::min(K2, t1 - t));
      if (st) return st;
    }
    const int64_t nsub = (t1 - t0 + K2 - 1) / K2;
    for (int64_t u = nsub - 1; u >= 0; --u) {
      st = reverse_segment(h, t0 + u * K2, std::min(t1, t0 + u * K2 + K2),
                           (const char*)d_mid + (size_t)u * bytes, d_seg, lam, &lc);
      if (st) return st;
    }
  }
  return backward_finish(h, d_ckpt, h_grad);
}

// ---------------------------------------------------------------- tiles
scd_status scd_tile_set(scd_lattice* h, int32_t variant, int32_t zc) {
  if (!h) return fail(SCD_EINVAL, "NULL handle");
  if (variant < 0 || variant >= variant_count())
    return fail(SCD_EINVAL, "variant %d is not compiled", variant);
  if (zc < 1) return fail(SCD_EINVAL, "z-chunk must be >= 1");
  h->variant = variant;
  h->zc = std::min<int32_t>(zc, h->p.nz);
  drop_graph(h);
  return SCD_OK;
}

scd_status scd_tile_get(const scd_lattice* h, int32_t* variant, int32_t* zc) {
  if (!h || !variant || !zc) return fail(SCD_EINVAL, "NULL argument");
  *variant = h->variant;
  *zc = h->zc;
  return SCD_OK;
}

scd_status scd_tile_list(int32_t* rows, int32_t cap, int32_t* n) {
  if (!n) return fail(SCD_EINVAL, "NULL argument");
  const int cnt = variant_count();
  for (int i = 0; i < cnt && i < cap; ++i)
    variant_at(i, &rows[4 * i], &rows[4 * i + 1], &rows[4 * i + 2], &rows[4 * i + 3]);
  *n = cnt;
  return SCD_OK;
}

static std::string device_name() {
  int dev = 0;
  (void)hipGetDevice(&dev);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  return std::string(prop.gcnArchName);
}

static std::string tune_key(const scd_lattice* h) {
  std::ostringstream o;
  o << h->p.nx << "x" << h->p.ny << "x" << h->p.nz << ":" << (h->p.dtype == SCD_F64 ? "f64" : "f32")
    << ":" << device_name() << ":v" << variant_count();
  return o.str();
}

// The last line of the JSON-lines cache whose key matches: "best": [a, b, c].
static bool cache_lookup3(const char* path, const std::string& key, int* best, double* ms) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  const std::string k = "\"key\": \"" + key + "\"";
  while (std::getline(f, line)) {
    if (line.find(k) == std::string::npos) continue;
    int a, c, d;
    double t;
    const char* s = strstr(line.c_str(), "\"best\": [");
    const char* m = strstr(line.c_str(), "\"ms\": ");
    if (!s || !m) continue;
    if (sscanf(s, "\"best\": [%d, %d, %d]", &a, &c, &d) == 3 && sscanf(m, "\"ms\": %lf", &t) == 1) {
      best[0] = a;
      best[1] = c;
      best[2] = d;
      *ms = t;
      found = true;
    }
  }
  return found;
}

static bool cache_lookup(const char* path, const std::string& key, int* best, double* ms) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    const std::string k = "\"key\": \"" + key + "\"";
    if (line.find(k) == std::string::npos) continue;
    int v, zc;
    double t;
    const char* s = strstr(line.c_str(), "\"best\": [");
    const char* m = strstr(line.c_str(), "\"ms\": ");
    if (!s || !m) continue;
    if (sscanf(s, "\"best\": [%d, %d]", &v, &zc) == 2 && sscanf(m, "\"ms\": %lf", &t) == 1) {
      best[0] = v;
      best[1] = zc;
      *ms = t;
      found = true;  // the last matching line wins
    }
  }
  return found;
}

scd_status scd_autotune(scd_lattice* h, int32_t steps_per_trial, const char* cache_path,
                        int32_t* best, double* best_ms) {
  TraceRange trace_("scd_autotune");
  if (!h || !best || !best_ms) return fail(SCD_EINVAL, "NULL argument");
  if (steps_per_trial < 2) return fail(SCD_EINVAL, "steps_per_trial must be >= 2");
  const std::string key = tune_key(h);
  int cached[2];
  double cms;
  if (cache_lookup(cache_path, key, cached, &cms) && cached[0] >= 0 && cached[0] < variant_count()) {
    scd_status st = scd_tile_set(h, cached[0], cached[1]);
    if (st) return st;
    best[0] = cached[0];
    best[1] = cached[1];
    *best_ms = cms;
    return SCD_OK;
  }
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  double bms = 1e30;
  int b[2] = {h->variant, h->zc};
  for (int i = 0; i < variant_count(); ++i) {
    int tx, ty, var, wpe;
    variant_at(i, &tx, &ty, &var, &wpe);
    if (tx > 2 * h->p.nx && tx > 16) continue;  // mostly idle lanes
    // powers of two and the chunk the wave-count model picks for this variant
    const int zcs[] = {4, 8, 16, 32, 64, 128, default_zc(h->p, i)};
    for (int zi = 0; zi < 7; ++zi) {
      const int zc = zcs[zi];
      if (zc > h->p.nz && zc != zcs[0]) continue;
      if (zi == 6 && (zc & (zc - 1)) == 0 && zc <= 128) continue;  // already timed
      scd_status st = scd_tile_set(h, i, zc);
      if (st) return st;
      st = enqueue_steps(h, 1);  // warm-up
      if (st) return st;
      HIPCHK(hipEventRecord(e0, h->stream));
      st = enqueue_steps(h, steps_per_trial);
      if (st) return st;
      HIPCHK(hipEventRecord(e1, h->stream));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      const double per = ms / steps_per_trial;
      if (per < bms) {
        bms = per;
        b[0] = i;
        b[1] = std::min(zc, h->p.nz);
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  scd_status st = scd_tile_set(h, b[0], b[1]);
  if (st) return st;
  best[0] = b[0];
  best[1] = b[1];
  *best_ms = bms;
  if (cache_path) {
    std::ofstream f(cache_path, std::ios::app);
    f << "{\"key\": \"" << key << "\", \"best\": [" << b[0] << ", " << b[1]
      << "], \"ms\": " << std::setprecision(17) << bms << "}\n";
  }
  return SCD_OK;
}

// ---------------------------------------------------------------- graphs
scd_status scd_graph_capture(scd_lattice* h, int64_t nsteps) {
  if (!h) return fail(SCD_EINVAL, "NULL handle");
  if (nsteps < 2 || (nsteps & 1)) return fail(SCD_EINVAL, "graph step count must be even and > 0");
  if (!h->stream) return fail(SCD_EINVAL, "graph capture needs a non-default stream");
  drop_graph(h);
  const int cur0 = h->cur;
  const int64_t step0 = h->step;
  HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  scd_status st = enqueue_steps(h, nsteps);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(h->stream, &g);
  h->cur = cur0;  // capture does not run anything
  h->step = step0;
  if (st) return st;
  if (e != hipSuccess) return fail(SCD_EDEVICE, "capture: %s", hipGetErrorString(e));
  h->graph = g;
  HIPCHK(hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0));
  h->graph_steps = nsteps;
  h->graph_cur = cur0;
  return SCD_OK;
}

scd_status scd_graph_replay(scd_lattice* h, int64_t reps) {
  TraceRange trace_("scd_graph_replay");
  if (!h) return fail(SCD_EINVAL, "NULL handle");
  if (!h->gexec) return fail(SCD_EINVAL, "no captured graph");
  if (h->cur != h->graph_cur) return fail(SCD_EINVAL, "buffer parity changed since capture");
  for (int64_t r = 0; r < reps; ++r) {
    HIPCHK(hipGraphLaunch(h->gexec, h->stream));
    h->step += h->graph_steps;
  }
  return SCD_OK;
}

}  // extern "C"

// ======================================================================= batch
struct scd_batch {
  int n;
  int dtype;
  std::vector<scd_lattice*> views;
  char* arena;
  std::vector<char> desc[2];  // host descriptors of every member, even and odd parity
  int nitems;
  int variant, zc, grid;  // the last uniform setting (scd_batch_set_tile)
  int remap;              // XCD-contiguous ranges of the work list
  std::vector<int> mvar, mzc;  // per member: step variant and z-chunk
  int64_t set_bytes;           // cache-blocking budget (0: one set)
  int nsets;
  struct Group {
    int set, variant, count;   // members of one set and variant: one launch per step
    std::vector<int> members;  // at most BATCH_DESC_MAX
    std::vector<int> geo;      // per member: tile columns along x, chunks per column, chunk length
  };
  std::vector<Group> groups;
  hipStream_t stream;
  int parity;
  hipGraph_t graph;
  hipGraphExec_t gexec;
  int64_t graph_steps;
  int graph_parity;
};

namespace {

struct BatchLayout {
  std::vector<size_t> pop0, pop1, work;
  size_t total;
};

BatchLayout batch_layout(int n, const scd_params* p) {
  BatchLayout L;
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    size_t pb, wb;
    scd_sizes(&p[i], &pb, &wb);
    L.pop0.push_back(off); off += align256(pb);
    L.pop1.push_back(off); off += align256(pb);
    L.work.push_back(off); off += align256(wb);
  }
  L.total = off;
  return L;
}

// Bytes a member's step streams through: both population buffers and the
// link masks.
size_t member_state_bytes(const scd_lattice* v) {
  size_t pb = 0;
  (void)scd_sizes(&v->p, &pb, nullptr);
  return 2 * pb + v->N * sizeof(uint32_t);
}

scd_status batch_upload(scd_batch* b) {
  // descriptors for both parities and the launch groups.  The members are
  // packed, in index order, into sets of at most set_bytes of state; within
  // a set they are taken in order of their step variant, and the members of
  // one set and variant form launch groups of at most BATCH_DESC_MAX (one
  // launch per group and step).  A member's items, (tile column, z-chunk)
  // pairs, are numbered as in the single-lattice step.
  const size_t ds = latdev_size(b->dtype);
  std::vector<char>& d0 = b->desc[0];
  std::vector<char>& d1 = b->desc[1];
  d0.assign(ds * b->n, 0);
  d1.assign(ds * b->n, 0);
  std::vector<int> order(b->n), mset(b->n);
  {
    int s = 0;
    size_t acc = 0;
    for (int i = 0; i < b->n; ++i) {
      const size_t fb = member_state_bytes(b->views[i]);
      if (b->set_bytes > 0 && acc > 0 && acc + fb > (size_t)b->set_bytes) {
        ++s;
        acc = 0;
      }
      mset[i] = s;
      acc += fb;
    }
    b->nsets = s + 1;
  }
  for (int i = 0; i < b->n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return mset[x] != mset[y] ? mset[x] < mset[y] : b->mvar[x] < b->mvar[y];
  });
  b->groups.clear();
  for (int i = 0; i < b->n; ++i) {
    scd_lattice* v = b->views[i];
    latdev_fill(b->dtype, d0.data() + ds * i, v->pop[0], v->pop[1], v->links(), v->p.nx, v->p.ny,
                v->p.nz, v->ph);
    latdev_fill(b->dtype, d1.data() + ds * i, v->pop[1], v->pop[0], v->links(), v->p.nx, v->p.ny,
                v->p.nz, v->ph);
  }
  int64_t total = 0;
  for (int i : order) {
    scd_lattice* v = b->views[i];
    const int zc = std::min(b->mzc[i], v->p.nz);
    int tx, ty, var, wpe;
    variant_at(b->mvar[i], &tx, &ty, &var, &wpe);
    const int gx = (v->p.nx + tx - 1) / tx, gy = (v->p.ny + ty - 1) / ty;
    const int gz = (v->p.nz + zc - 1) / zc;
    if (b->groups.empty() || b->groups.back().variant != b->mvar[i] || b->groups.back().set != mset[i] ||
        (int)b->groups.back().members.size() == BATCH_DESC_MAX)
      b->groups.push_back({mset[i], b->mvar[i], 0, {}, {}});
    scd_batch::Group& g = b->groups.back();
    const int64_t items = (int64_t)gx * gy * gz;
    if (g.count + items > INT32_MAX / 2) return fail(SCD_EINVAL, "too many tiles in one launch group");
    g.members.push_back(i);
    g.geo.insert(g.geo.end(), {gx, gz, zc});
    g.count += (int)items;
    total += items;
  }
  b->nitems = (int)std::min<int64_t>(total, INT32_MAX);
  return SCD_OK;
}

// Default batch tile: with many (lattice, tile) items the z-halo re-reads of
// short chunks cost more than the lost parallelism of long ones, so the
// batch marches 32 planes per item with the single-lattice default variant;
// one workgroup per item (grid 0), items dealt to the XCDs in contiguous
// ranges.
void batch_default_tile(int dtype, int* variant, int* zc, int* grid) {
  *variant = default_variant(dtype);
  *zc = 32;
  *grid = 0;
}

void batch_drop_graph(scd_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  b->graph_steps = 0;
}

scd_status batch_enqueue(scd_batch* b, int64_t nsteps) {
  // set by set, every step of the call: the members of one set are stepped
  // nsteps times before the next set starts (members are independent, so
  // the order changes no result).  Per step, one launch per variant group:
  // one workgroup per item, or a persistent grid (a multiple of 8 with the
  // XCD remap, so that each block stays on one XCD's range)
  size_t g0 = 0;
  while (g0 < b->groups.size()) {
    size_t g1 = g0;
    while (g1 < b->groups.size() && b->groups[g1].set == b->groups[g0].set) ++g1;
    for (int64_t s = 0; s < nsteps; ++s) {
      const int par = b->parity ^ (int)(s & 1);
      for (size_t gi = g0; gi < g1; ++gi) {
        const auto& g = b->groups[gi];
        if (g.members.size() == 1 && b->grid <= 0) {
          // a group of one lattice, one workgroup per item, is the
          // single-lattice launch: the same kernel scd_step runs
          scd_lattice* v = b->views[g.members[0]];
          HIPCHK(launch_step(b->dtype, v->pop[par], v->pop[1 - par], v->links(), v->p.nx, v->p.ny,
                             v->p.nz, v->ph, g.variant, g.geo[2], b->remap, b->stream));
          continue;
        }
        const int slots = b->remap ? 8 * ((g.count + 7) / 8) : g.count;
        int grid = (b->grid <= 0 || b->grid > slots) ? slots : b->grid;
        if (b->remap) grid = 8 * ((grid + 7) / 8);
        // the group's descriptors for this parity, passed by value
        char descs[BATCH_DESC_MAX * 256];
        const size_t ds = latdev_size(b->dtype);
        if (ds > 256) return fail(SCD_EINVAL, "lattice descriptor larger than expected");
        for (size_t m = 0; m < g.members.size(); ++m)
          memcpy(descs + m * ds, b->desc[par].data() + (size_t)g.members[m] * ds, ds);
        HIPCHK(launch_step_batch(b->dtype, descs, (int)g.members.size(), g.geo.data(), grid,
                                 g.variant, b->remap, b->stream));
      }
    }
    g0 = g1;
  }
  b->parity ^= (int)(nsteps & 1);
  for (scd_lattice* v : b->views) {
    v->cur = b->parity;
    v->step += nsteps;
  }
  return SCD_OK;
}

}  // namespace

extern "C" {

scd_status scd_batch_sizes(int32_t n, const scd_params* p, size_t* arena_bytes) {
  if (n < 1 || !p || !arena_bytes) return fail(SCD_EINVAL, "bad batch arguments");
  for (int i = 0; i < n; ++i) {
    scd_status st = validate(&p[i]);
    if (st) return st;
    if (p[i].dtype != p[0].dtype) return fail(SCD_EINVAL, "all lattices of a batch share one dtype");
  }
  *arena_bytes = batch_layout(n, p).total;
  return SCD_OK;
}

scd_status scd_batch_create(int32_t n, const scd_params* p, const uint8_t* const* d_solid,
                            void* d_arena, void* stream, scd_batch** out) {
  size_t bytes;
  scd_status st = scd_batch_sizes(n, p, &bytes);
  if (st) return st;
  if (!d_solid || !d_arena || !out) return fail(SCD_EINVAL, "NULL argument");
  if ((uintptr_t)d_arena & 255) return fail(SCD_EINVAL, "arena must be 256-byte aligned");
  BatchLayout L = batch_layout(n, p);
  scd_batch* b = new scd_batch();
  b->n = n;
  b->dtype = p[0].dtype;
  b->arena = (char*)d_arena;
  batch_default_tile(p[0].dtype, &b->variant, &b->zc, &b->grid);
  b->remap = 1;
  b->set_bytes = 0;
  b->nsets = 1;
  b->mvar.assign(n, b->variant);
  b->mzc.assign(n, b->zc);
  b->stream = (hipStream_t)stream;
  b->parity = 0;
  b->graph = nullptr;
  b->gexec = nullptr;
  b->graph_steps = 0;
  b->graph_parity = 0;
  for (int i = 0; i < n; ++i) {
    scd_lattice* v = nullptr;
    st = scd_create(&p[i], d_solid[i], b->arena + L.pop0[i], b->arena + L.pop1[i],
                    b->arena + L.work[i], stream, &v);
    if (st) {
      for (scd_lattice* w : b->views) scd_destroy(w);
      delete b;
      return st;
    }
    v->batch_view = true;
    b->views.push_back(v);
  }
  st = batch_upload(b);
  if (st) {
    for (scd_lattice* w : b->views) scd_destroy(w);
    delete b;
    return st;
  }
  *out = b;
  return SCD_OK;
}

scd_status scd_batch_destroy(scd_batch* b) {
  if (!b) return SCD_OK;
  batch_drop_graph(b);
  for (scd_lattice* v : b->views) scd_destroy(v);
  delete b;
  return SCD_OK;
}

scd_status scd_batch_lattice(scd_batch* b, int32_t i, scd_lattice** view) {
  if (!b || !view || i < 0 || i >= b->n) return fail(SCD_EINVAL, "bad batch index");
  *view = b->views[i];
  return SCD_OK;
}

scd_status scd_batch_init_equilibrium(scd_batch* b, int32_t i, const double* d_rho_a,
                                      const double* d_rho_b) {
  if (!b || i < 0 || i >= b->n) return fail(SCD_EINVAL, "bad batch index");
  scd_lattice* v = b->views[i];
  v->cur = b->parity;
  return scd_init_equilibrium(v, d_rho_a, d_rho_b);
}

scd_status scd_batch_set_tile(scd_batch* b, int32_t variant, int32_t zc, int32_t grid) {
  if (!b) return fail(SCD_EINVAL, "NULL handle");
  if (variant < 0 || variant >= variant_count())
    return fail(SCD_EINVAL, "variant %d is not compiled", variant);
  if (zc < 1 || zc > 32767 || grid < 0)
    return fail(SCD_EINVAL, "z-chunk must be in [1, 32767] and grid >= 0");
  b->variant = variant;
  b->zc = zc;
  b->grid = grid;
  b->mvar.assign(b->n, variant);
  b->mzc.assign(b->n, zc);
  for (scd_lattice* v : b->views) { v->variant = variant; v->zc = std::min(zc, v->p.nz); }
  batch_drop_graph(b);
  return batch_upload(b);
}

scd_status scd_batch_set_member_tile(scd_batch* b, int32_t i, int32_t variant, int32_t zc) {
  if (!b || i < 0 || i >= b->n) return fail(SCD_EINVAL, "bad batch index");
  if (variant < 0 || variant >= variant_count())
    return fail(SCD_EINVAL, "variant %d is not compiled", variant);
  if (zc < 1 || zc > 32767) return fail(SCD_EINVAL, "z-chunk must be in [1, 32767]");
  b->mvar[i] = variant;
  b->mzc[i] = zc;
  b->views[i]->variant = variant;
  b->views[i]->zc = std::min(zc, b->views[i]->p.nz);
  batch_drop_graph(b);
  return batch_upload(b);
}

scd_status scd_batch_member_tile(const scd_batch* b, int32_t i, int32_t* variant, int32_t* zc) {
  if (!b || i < 0 || i >= b->n || !variant || !zc) return fail(SCD_EINVAL, "bad argument");
  *variant = b->mvar[i];
  *zc = b->mzc[i];
  return SCD_OK;
}

scd_status scd_batch_step(scd_batch* b, int64_t nsteps) {
  TraceRange trace_("scd_batch_step");
  if (!b) return fail(SCD_EINVAL, "NULL handle");
  if (nsteps < 0) return fail(SCD_EINVAL, "nsteps < 0");
  return batch_enqueue(b, nsteps);
}

scd_status scd_batch_graph_capture(scd_batch* b, int64_t nsteps) {
  if (!b) return fail(SCD_EINVAL, "NULL handle");
  if (nsteps < 2 || (nsteps & 1)) return fail(SCD_EINVAL, "graph step count must be even and > 0");
  if (!b->stream) return fail(SCD_EINVAL, "graph capture needs a non-default stream");
  batch_drop_graph(b);
  const int par0 = b->parity;
  std::vector<int64_t> steps0;
  for (scd_lattice* v : b->views) steps0.push_back(v->step);
  HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  scd_status st = batch_enqueue(b, nsteps);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->stream, &g);
  b->parity = par0;
  for (int i = 0; i < b->n; ++i) { b->views[i]->cur = par0; b->views[i]->step = steps0[i]; }
  if (st) return st;
  if (e != hipSuccess) return fail(SCD_EDEVICE, "capture: %s", hipGetErrorString(e));
  b->graph = g;
  HIPCHK(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
  b->graph_steps = nsteps;
  b->graph_parity = par0;
  return SCD_OK;
}

// A named integer list (or, with one element, a number) of the last line
// of a cached batch tuning whose key matches (empty when there is none).
static std::vector<long long> cache_list(const char* path, const std::string& key, const char* name) {
  std::vector<long long> out;
  if (!path) return out;
  std::ifstream f(path);
  std::string line;
  const std::string k = "\"key\": \"" + key + "\"";
  const std::string field = std::string("\"") + name + "\": ";
  while (std::getline(f, line)) {
    if (line.find(k) == std::string::npos) continue;
    const size_t at = line.find(field);
    if (at == std::string::npos) continue;
    std::vector<long long> v;
    const char* c = line.c_str() + at + field.size();
    const bool list = *c == '[';
    if (list) ++c;
    while (*c && *c != ']') {
      char* e = nullptr;
      const long long x = strtoll(c, &e, 10);
      if (e == c) break;
      v.push_back(x);
      c = e;
      if (!list) break;
      while (*c == ',' || *c == ' ') ++c;
    }
    out = v;
  }
  return out;
}

scd_status scd_batch_autotune(scd_batch* b, int32_t steps_per_trial, const char* cache_path,
                              int32_t* best, double* best_ms) {
  TraceRange trace_("scd_batch_autotune");
  if (!b || !best || !best_ms) return fail(SCD_EINVAL, "NULL argument");
  if (steps_per_trial < 2) return fail(SCD_EINVAL, "steps_per_trial must be >= 2");
  // key: member count, a hash of the member shapes, dtype, device, variant count
  uint64_t hsh = 1469598103934665603ull;
  for (scd_lattice* v : b->views)
    for (int d : {v->p.nx, v->p.ny, v->p.nz}) hsh = (hsh ^ (uint64_t)d) * 1099511628211ull;
  std::ostringstream ko;
  ko << "batch" << b->n << ":" << std::hex << hsh << std::dec << ":" << (b->dtype == SCD_F64 ? "f64" : "f32")
     << ":" << device_name() << ":v" << variant_count() << ":sets";
  const std::string key = ko.str();

  // members' variants and chunks (zc 0: each member's model chunk), grid and
  // set budget, applied and uploaded
  auto apply = [&](const std::vector<int>& mv, const std::vector<int>& mz, int grid,
                   int64_t sb) -> scd_status {
    b->mvar = mv;
    b->mzc = mz;
    b->grid = grid;
    b->set_bytes = sb;
    for (int i = 0; i < b->n; ++i) {
      b->views[i]->variant = mv[i];
      b->views[i]->zc = std::min(mz[i], b->views[i]->p.nz);
    }
    batch_drop_graph(b);
    return batch_upload(b);
  };
  auto chunks = [&](const std::vector<int>& mv, int zc) {
    std::vector<int> mz(b->n);
    for (int i = 0; i < b->n; ++i) mz[i] = zc > 0 ? zc : default_zc(b->views[i]->p, mv[i]);
    return mz;
  };
  auto summary = [&](const std::vector<int>& mv, const std::vector<int>& mz) {
    int cnt[64] = {0}, top = mv[0];
    for (int x : mv)
      if (x < 64 && ++cnt[x] > cnt[top]) top = x;
    bool same = true;
    for (int z : mz) same = same && z == mz[0];
    b->variant = top;
    b->zc = same ? mz[0] : 0;
  };

  {
    int cached[3];
    double cms;
    if (cache_lookup3(cache_path, key, cached, &cms) && cached[0] >= 0 && cached[0] < variant_count()) {
      const std::vector<long long> mv = cache_list(cache_path, key, "members");
      const std::vector<long long> mz = cache_list(cache_path, key, "zcs");
      const std::vector<long long> sb = cache_list(cache_path, key, "set_bytes");
      if ((int)mv.size() == b->n && (int)mz.size() == b->n && sb.size() == 1 && sb[0] >= 0) {
        std::vector<int> v(b->n), z(b->n);
        for (int i = 0; i < b->n; ++i) {
          if (mv[i] < 0 || mv[i] >= variant_count()) return fail(SCD_EINVAL, "bad cached variant %lld", mv[i]);
          if (mz[i] < 1 || mz[i] > 32767) return fail(SCD_EINVAL, "bad cached z-chunk %lld", mz[i]);
          v[i] = (int)mv[i];
          z[i] = (int)mz[i];
        }
        scd_status st = apply(v, z, cached[2], sb[0]);
        if (st) return st;
        summary(v, z);
        for (int j = 0; j < 3; ++j) best[j] = cached[j];
        *best_ms = cms;
        return SCD_OK;
      }
    }
  }
  const int cus = device_cus();
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  auto time_batch = [&](double* per) -> scd_status {
    scd_status st = batch_enqueue(b, 1);  // warm-up
    if (st) return st;
    HIPCHK(hipEventRecord(e0, b->stream));
    st = batch_enqueue(b, steps_per_trial);
    if (st) return st;
    HIPCHK(hipEventRecord(e1, b->stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    *per = ms / steps_per_trial;
    return SCD_OK;
  };
  double bms = 1e30;
  std::vector<int> bmem = b->mvar, bzc = b->mzc;  // the current tiles until a trial beats them
  int bgrid = 0;
  int64_t bsb = 0;
  auto trial = [&](const std::vector<int>& mv, const std::vector<int>& mz, int grid,
                   int64_t sb) -> scd_status {
    scd_status st = apply(mv, mz, grid, sb);
    if (st) return st;
    double per;
    st = time_batch(&per);
    if (st) return st;
    if (per < bms) {
      bms = per;
      bmem = mv;
      bzc = mz;
      bgrid = grid;
      bsb = sb;
    }
    return SCD_OK;
  };
  // (1) one variant for all members, all members in one set: every compiled
  // variant at 16- and 32-plane chunks, one workgroup per item
  for (int i = 0; i < variant_count(); ++i)
    for (int zc : {16, 32}) {
      const std::vector<int> mv(b->n, i);
      scd_status st = trial(mv, chunks(mv, zc), 0, 0);
      if (st) return st;
    }
  // (2) a tile per member: the fastest variant and z-chunk on the member
  // stepped alone (each variant at the wave-count model's chunk for that
  // lattice and at 4, 8, 16, 32 and 64 planes, over an even number of steps,
  // so that the member keeps the batch's buffer parity); then those tiles,
  // and those variants at one chunk for all, in one set, with both grids
  const int even = 2 * ((steps_per_trial + 1) / 2);
  std::vector<int> mv(b->n), mz(b->n);
  for (int m = 0; m < b->n; ++m) {
    scd_lattice* v = b->views[m];
    double best_t = 1e30;
    mv[m] = bmem[m];
    mz[m] = std::min(bzc[m], v->p.nz);
    for (int i = 0; i < variant_count(); ++i) {
      int tx, ty, var, wpe;
      variant_at(i, &tx, &ty, &var, &wpe);
      if (tx > 2 * v->p.nx && tx > 16) continue;  // mostly idle lanes
      const int model = default_zc(v->p, i);
      for (int zc : {model, 4, 8, 16, 32, 64}) {
        const int z = std::min(zc, v->p.nz);
        if (zc != model && z == std::min(model, v->p.nz)) continue;  // timed already
        v->variant = i;
        v->zc = z;
        scd_status st = enqueue_steps(v, 2);
        if (st) return st;
        HIPCHK(hipEventRecord(e0, b->stream));
        st = enqueue_steps(v, even);
        if (st) return st;
        HIPCHK(hipEventRecord(e1, b->stream));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_t) {
          best_t = ms;
          mv[m] = i;
          mz[m] = z;
        }
      }
    }
  }
  for (int grid : {0, 4 * cus}) {
    scd_status st = trial(mv, mz, grid, 0);
    if (st) return st;
    for (int zc : {0, 8, 16, 32, 48, 64}) {
      st = trial(mv, chunks(mv, zc), grid, 0);
      if (st) return st;
    }
  }
  // (3) cache blocking: sets of at most 64, 128, 192 or 256 MiB of state, or
  // every member alone, with the best so far and with the per-member tiles
  {
    const std::vector<int> m0 = bmem, z0 = bzc;
    const int g0 = bgrid;
    for (int64_t mib : {64, 128, 192, 256, 0}) {
      const int64_t sb = mib ? mib << 20 : 1;
      scd_status st = trial(m0, z0, g0, sb);
      if (st) return st;
      st = trial(mv, mz, 0, sb);
      if (st) return st;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // apply the fastest
  scd_status st = apply(bmem, bzc, bgrid, bsb);
  if (st) return st;
  summary(bmem, bzc);
  best[0] = b->variant;
  best[1] = b->zc;
  best[2] = bgrid;
  *best_ms = bms;
  if (cache_path) {
    std::ofstream f(cache_path, std::ios::app);
    f << "{\"key\": \"" << key << "\", \"best\": [" << best[0] << ", " << best[1] << ", " << best[2]
      << "], \"members\": [";
    for (int i = 0; i < b->n; ++i) f << (i ? ", " : "") << bmem[i];
    f << "], \"zcs\": [";
    for (int i = 0; i < b->n; ++i) f << (i ? ", " : "") << bzc[i];
    f << "], \"set_bytes\": " << bsb << ", \"ms\": " << std::setprecision(17) << bms << "}\n";
  }
  return SCD_OK;
}

scd_status scd_batch_set_blocking(scd_batch* b, int64_t set_bytes) {
  if (!b) return fail(SCD_EINVAL, "NULL handle");
  if (set_bytes < 0) return fail(SCD_EINVAL, "set_bytes < 0");
  b->set_bytes = set_bytes;
  batch_drop_graph(b);
  return batch_upload(b);
}

scd_status scd_batch_blocking(const scd_batch* b, int64_t* set_bytes, int32_t* nsets) {
  if (!b || !set_bytes || !nsets) return fail(SCD_EINVAL, "NULL argument");
  *set_bytes = b->set_bytes;
  *nsets = b->nsets;
  return SCD_OK;
}

scd_status scd_batch_graph_replay(scd_batch* b, int64_t reps) {
  TraceRange trace_("scd_batch_graph_replay");
  if (!b) return fail(SCD_EINVAL, "NULL handle");
  if (!b->gexec) return fail(SCD_EINVAL, "no captured graph");
  if (b->parity != b->graph_parity) return fail(SCD_EINVAL, "buffer parity changed since capture");
  for (int64_t r = 0; r < reps; ++r) {
    HIPCHK(hipGraphLaunch(b->gexec, b->stream));
    for (scd_lattice* v : b->views) v->step += b->graph_steps;
  }
  return SCD_OK;
}

}  // extern "C"
