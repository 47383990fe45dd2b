// kp_internal.hpp -- records shared by the host API and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kp {

// Per-wavelength constants, prepared on the host from kp_dust.
struct DustDev {
  double ks_cell;    // kappa_sca * dx   (per unit density, per cell length)
  double ka_cell;    // kappa_abs * dx
  double ke_cell;    // (kappa_sca + kappa_abs) * dx
  double kext;       // kappa_sca + kappa_abs (per unit length)
  double ap_re, ap_im, aa_re, aa_im;
  double inv2cavg;   // 1 / (2 C_avg), C_avg = (2 Im a_perp + Im a_par)/3
  double alpha3_scale;
  double pfac;       // 3 / (8 pi N_P),  N_P = (2|a_perp|^2 + |a_par|^2)/3
  double bound_fac;  // pfac * max(|a_perp|^2, |a_par|^2)
  double ap2_np, aa2_np;  // |a_perp|^2 / N_P, |a_par|^2 / N_P
  double w0;         // lum / N_lambda
  uint64_t first;    // first global work index of this wavelength
  uint64_t count;    // packets of this wavelength
  int32_t sphere;
  int32_t tab_n;     // tabulated scattering: nodes (0 = dipole grains)
  // tabulated scattering (device arrays): the scattering-plane elements S11
  // S12 S22 S33 S34 S44 divided by 2 pi times the integral of S11 over cos
  // Theta [tab_n][6], cos Theta at the nodes [tab_n] (Theta uniform on
  // [0, pi]), and the cumulative envelope mass [tab_n] (cum[j+1] - cum[j] =
  // max(S11_j, S11_j+1) (mu_j - mu_j+1), normalised elements)
  const double* tab;
  const double* tab_mu;
  const double* tab_cum;
  // guide to the node interval of a cos Theta: [tab_g] over cos Theta uniform
  // on [-1, 1] from 1 down, entry b the interval holding 1 - 2 b / tab_g
  const int32_t* tab_guide;
  int32_t tab_g;
  int32_t pad2;
};

struct ViewDev {
  double ox, oy, oz;     // camera direction
  double tx, ty, tz;     // theta_hat
  double px, py, pz;     // phi_hat
  double half_width;
};

struct StatsDev {
  unsigned long long cell_steps, scatterings, trials, rr_kills, rr_survivals, escaped,
      budget, numeric, packets, tally_flushes;
  double e_emitted, e_escaped, e_absorbed, e_rr_killed, e_rr_gained, e_budget, e_scat_delta;
};

struct TraceDev {
  uint64_t packet;
  int32_t end_kind;
  int32_t events;
  int64_t steps;
  int64_t last_cell;
  double n[3];
  double stokes[4];
  uint64_t hash;
  double tau_path;
};

// Composite mesh with static refinement (device view): root blocks of
// block^3 cells on an rx*ry*rz array, each the root of a tree of blocks split
// into octants; cells of leaf j have flat indices j*block^3 + local (x
// fastest).  Positions in units of the finest cell (2^-max_level of a root
// cell) locate leaves.
struct MeshDev {
  const int32_t* child;         // [n_nodes]: -1 leaf, else the first of 8 children
  const int32_t* leaf_of_node;  // [n_nodes]: leaf id or -1
  const int32_t* leaf_org;      // [n_leaves][4]: lower corner (finest cells), level
  int rx, ry, rz, block, max_level;
  int nfine[3];                 // domain extent in finest cells
  double fine;                  // finest cell edge
};

// a packet ends as an event-cap packet after this many cell steps (one that
// cannot scatter and moves parallel to every open face of a partly periodic
// grid would never leave it); camera rays longer than this many cells are
// refused
constexpr int KP_MAX_STEPS = 1 << 24;

struct TransportArgs {
  const float* rho;
  const float* bx;
  const float* by;
  const float* bz;
  int nx, ny, nz;
  double x0, y0, z0, dx;
  const DustDev* dust;
  int n_lambda;
  uint64_t total;
  int src_kind;
  double sx, sy, sz;
  double dx_, dy_, dz_;  // pencil direction (unit)
  uint64_t seed;
  double rr_wmin, rr_psurv;
  int max_events;
  double* tally;  // [lambda][nslot][stride] coherency blocks, or for tabulated
                  // grains the per-view source [lambda][nslot][view][4], cells
                  // at their tally_slot
  uint64_t ncell;
  uint64_t nslot;  // tally slots per wavelength (tally_slots; ncell on a mesh)
  int tbx, tby;    // bricks along x and y of the tally layout (0 on a mesh)
  unsigned long long* counter;
  StatsDev* stats;
  TraceDev* traces;
  uint32_t trace_count, trace_stride;
  int scatter_batch;  // run parked scattering events once this many lanes wait
  int scatter_wait;   // ... or after this many iterations
  // thermal emission of the dust (src_kind 2): per wavelength the running
  // sum of cell luminosities [lambda][ncell] and its guide table
  // [lambda][ncell + 1] (entry k: the first cell whose running sum exceeds
  // L k / ncell; entry ncell: the last cell)
  const double* em_cdf;
  const uint32_t* em_guide;
  int boundary;          // bit a: axis a periodic
  // cameras (peel-off imaging, and the per-view source of tabulated grains)
  // and the peel-off images [lambda][view][4][npy][npx] the scattering events
  // are added to (the kernels instantiated with peel-off)
  const ViewDev* views;
  int n_views, npx, npy;
  double* peel;
  MeshDev mesh;          // the kernels instantiated for a composite mesh
};

struct ImageArgs {
  const float* rho;
  const float* bx;
  const float* by;
  const float* bz;
  int nx, ny, nz;
  double x0, y0, z0, dx;
  const DustDev* dust;
  const ViewDev* views;
  int n_views, n_lambda, npx, npy;
  const double* tally;  // [lambda][nslot][stride] coherency source (tally layout)
  const double* user_S; // [lambda][nslot][view][4] per-view source (or null)
  double* images;       // [lambda][view][4][npy][npx]
  uint64_t ncell;
  uint64_t nslot;       // slots per wavelength of tally / user_S, and their
  int tbx, tby;         // bricks (tbx = 0: cell order, a caller's S or a mesh)
  const float* em_B;    // [lambda][ncell] source function of the dust's thermal
                        // emission, or null (no thermal source term)
  int boundary;         // bit a: axis a periodic
  MeshDev mesh;         // the kernels instantiated for a composite mesh
};

// Tally slot of cell c = (i, j, k) of a uniform grid: the tally and the
// per-view source are stored in bricks of 4 x 4 x 4 cells (bricks x-fastest
// over tbx x tby x .., cells x-fastest inside a brick), so that the flushes
// of a packet's successive cells, neighbours in space, fall in a few DRAM
// rows instead of rows 1 KB (y) and 256 KB (z) apart; on the 256^3 disk the
// flush rate rose from 1.61e10 to 1.85e10 lines/s.  tbx == 0 keeps the cell
// order (a composite mesh, whose leaf blocks are contiguous already, and a
// caller's source array).
__host__ __device__ inline uint64_t tally_slot(uint64_t c, int i, int j, int k, int tbx, int tby) {
  if (tbx == 0) return c;
  return ((((uint64_t)(k >> 2) * (uint64_t)tby + (uint64_t)(j >> 2)) * (uint64_t)tbx + (uint64_t)(i >> 2)) << 6) |
         (uint64_t)(((k & 3) << 4) | ((j & 3) << 2) | (i & 3));
}
// slots per wavelength of an nx x ny x nz grid in the brick layout
inline uint64_t tally_slots(int nx, int ny, int nz) {
  return 64ull * (uint64_t)((nx + 3) / 4) * (uint64_t)((ny + 3) / 4) * (uint64_t)((nz + 3) / 4);
}

// Tally layout [lambda][slot][stride] FP64: 6 reals (stride 8, one 64-B block
// per cell) when every wavelength has spherical grains, else 9 (stride 16).
// With stride 16 the slot after the coherency holds the cell's density and
// the next four the unit quaternion of its grain frame (read by the
// transport step from the same line its atomics update).
inline int tally_components(bool sphere) { return sphere ? 6 : 9; }
inline int tally_stride(bool sphere) { return sphere ? 8 : 16; }

// launchers (kp_kernels.hip)
hipError_t launch_transport(const TransportArgs& a, bool fp64, bool aligned, bool sphere, bool peel, bool tab,
                            bool mesh, int blocks, int block_size, hipStream_t s);
hipError_t launch_image(const ImageArgs& a, bool aligned, bool sphere, bool user_source, bool mesh,
                        hipStream_t s);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_tally_init(double* tally, const float* rho, const float* bx, const float* by,
                             const float* bz, uint64_t ncell, int n_lambda, bool sphere, uint64_t nslot, int nx,
                             int ny, int tbx, int tby, hipStream_t s);
hipError_t launch_validate(const float* rho, const float* bx, const float* by, const float* bz,
                           uint64_t n, unsigned long long* bad, hipStream_t s);
int transport_max_blocks_per_cu(bool fp64, bool aligned, bool sphere, bool peel, bool tab, bool mesh,
                                int block_size);
// Thermal emission tables of one wavelength: cdf [ncell], the running sum
// of fac rho B (fac = 4 pi kappa_abs dx^3; on a composite mesh, leaf_org
// non-null, times 2^-3 level of each cell's leaf, block3 cells per leaf) in
// flat cell order, and its guide table [ncell + 1]; `partial` holds
// emission_blocks(ncell) doubles of scratch.
hipError_t launch_emission_table(const float* rho, const float* B, double fac, const int32_t* leaf_org,
                                 uint64_t block3, uint64_t ncell, double* partial, double* cdf, uint32_t* guide,
                                 hipStream_t s);
uint64_t emission_blocks(uint64_t ncell);

}  // namespace kp
