// kernels.hpp -- host-callable launchers of libscdrop's kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.hpp"

namespace scd {

using PhysD = Phys<double>;

template <typename real>
inline Phys<real> phys_cast(const PhysD& d) {
  Phys<real> r;
  for (int a = 0; a < 2; ++a) {
    r.tau[a] = (real)d.tau[a];
    r.inv_tau[a] = (real)d.inv_tau[a];
    r.gw[a] = (real)d.gw[a];
    r.psiw[a] = (real)d.psiw[a];
    r.dpsiw[a] = (real)d.dpsiw[a];
  }
  r.gab = (real)d.gab;
  r.wa = (real)d.wa;
  r.wd = (real)d.wd;
  r.psi_form = d.psi_form;
  return r;
}

// step.hip
hipError_t launch_links(const uint8_t* solid, uint32_t* links, int nx, int ny, int nz,
                        hipStream_t s);
hipError_t launch_init(int dtype, void* pop, const double* ra, const double* rb,
                       const uint32_t* links, int nx, int ny, int nz, hipStream_t s);
hipError_t launch_pop_repack(int dtype, const void* src, void* dst, int nx, int ny, int nz,
                             bool to_blocked, hipStream_t s);
hipError_t launch_density(int dtype, const void* pop, const uint32_t* links, double* rho, int nx,
                          int ny, int nz, hipStream_t s);
hipError_t launch_stream_density(int dtype, const void* pop, const uint32_t* links, void* rho,
                                 int nx, int ny, int nz, hipStream_t s);
hipError_t launch_fill(int dtype, void* p, size_t n, double v, hipStream_t s);
// mom_out (optional): the moments of the post-stream populations of src, 8
// fields of N (rho^A, rho^B, then j^A and j^B by component; rho is 0 at
// walls, j is left unwritten there), written by the variants for which
// variant_writes_moments holds.
hipError_t launch_step(int dtype, const void* src, void* dst, const uint32_t* links, int nx,
                       int ny, int nz, const PhysD& ph, int variant, int zc, int remap,
                       hipStream_t s, void* mom_out = nullptr);
bool variant_writes_moments(int variant);
// h_descs: ndesc (<= BATCH_DESC_MAX) lattice descriptors of latdev_size bytes
// each, and h_geo: per descriptor {tile columns along x, z-chunks per column,
// chunk length}, both on the host (passed by value); grid workgroups walk
// the members' (column, chunk) items (remap: XCD-contiguous ranges)
constexpr int BATCH_DESC_MAX = 16;
hipError_t launch_step_batch(int dtype, const void* h_descs, int ndesc, const int* h_geo, int grid,
                             int variant, int remap, hipStream_t s);
size_t latdev_size(int dtype);
void latdev_fill(int dtype, void* out, const void* src, void* dst, const uint32_t* links, int nx,
                 int ny, int nz, const PhysD& ph);
int variant_count();
void variant_at(int i, int* tx, int* ty, int* var, int* wpe);
int variant_find(int tx, int ty, int var, int wpe);

// observe.hip
constexpr int RED_BLOCKS = 512;   // blocks of the observable reductions
constexpr int RED_STRIDE = 8;     // doubles per block partial
// contact-angle result slots (doubles) in the work area
constexpr int CA_SLOTS = 32;
hipError_t launch_observables(int dtype, const void* pop, const uint32_t* links, int nx, int ny,
                              int nz, double* partials, double* result, hipStream_t s);
struct CaDev {
  int ic, jc, zs, off;
  double eps;
};
hipError_t launch_contact_angle(int dtype, const void* pop, const uint32_t* links, int nx, int ny,
                                int nz, CaDev cfg, double* phi_scratch, double* partials,
                                double* result, hipStream_t s);
hipError_t launch_pressure(int dtype, const void* pop, const uint32_t* links, int nx, int ny,
                           int nz, const PhysD& ph, void* rho, double* P, hipStream_t s);
hipError_t launch_radial(int dtype, const void* pop, const uint32_t* links, int nx, int ny, int nz,
                         const double* c, int periodic, int nbins, double* P, double* shells,
                         hipStream_t s);
hipError_t launch_plane_tension(int nx, int ny, int nz, const double* P, double* profile,
                                hipStream_t s);
hipError_t launch_stream_copy(const double* src, double* dst, size_t n, hipStream_t s);
hipError_t launch_pull_copy(int dtype, const void* src, const uint32_t* links, void* dst, int nx,
                            int ny, int nz, hipStream_t s);
// Largest plane (nx * ny) and depth the static contact-angle scratch holds,
// and the device address of that scratch on the current device (looked up
// once per device).
constexpr size_t CA_STATIC_MAX_PLANE = 512 * 512;
constexpr size_t CA_STATIC_MAX_NZ = 4096;
hipError_t ca_static_scratch(double** phi, double** partials, double** result);
hipError_t launch_ca_seed(int dtype, const uint32_t* links, int nx, int ny, int nz, CaDev cfg,
                          const double* phi_scratch, const double* result, double dL_dtheta,
                          void* lambda, hipStream_t s);

// adjoint.hip
constexpr int ADJ_BLOCKS = 8192;  // rows of adjoint partials (workgroups of the gathering pass, at most)
// One reverse step.  mom_cached (or nullptr): the moments of the post-stream
// populations of state_t in the layout of launch_step's mom_out, written
// earlier by the step that read state_t; the local pass then takes rho and j
// from them and pulls no populations.  Otherwise the densities are computed
// into rho_field and the moments from the pulled populations.  acc_partials == nullptr: this step's parameter gradient
// is summed into dparams_dev[0..5).  Otherwise the per-workgroup partials
// accumulate in acc_partials (ADJ_BLOCKS x RED_STRIDE doubles, zeroed by the
// caller) and launch_adjoint_sum reduces them when they are read.  Work
// fields: q_field 6 N, d_field 2 N and e_field 3 N reals (e = dL/du' / R,
// shared by both species); rho_field 2 N and j_field 6 N.
hipError_t launch_adjoint(int dtype, const void* state_t, const void* lam_in, void* lam_out,
                          const uint32_t* links, int nx, int ny, int nz, const PhysD& ph,
                          void* rho_field, void* j_field, const void* mom_cached, void* q_field,
                          void* d_field, void* e_field, double* partials, double* dparams_dev,
                          double* acc_partials, hipStream_t s);
hipError_t launch_adjoint_sum(int dtype, const double* partials, size_t N, double* out, hipStream_t s);
hipError_t launch_zero(double* p, int n, hipStream_t s);

}  // namespace scd
