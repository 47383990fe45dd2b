/*
 * polrad_oracle.h -- FP64 CPU oracle for polarized Monte Carlo radiative
 * transfer with two-step imaging (Yang & Wang, "Kratos-polrad").
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no source, header, table or helper with
 * the HIP library; the two agree only through the conventions written out in
 * the comments below (and restated independently in the HIP sources).
 *
 * Conventions (each one a reading of the paper, see polrad_oracle.c):
 *  - directions n = (sin t cos p, sin t sin p, cos t); Stokes reference basis
 *    theta_hat = (cos t cos p, cos t sin p, -sin t), phi_hat = (-sin p, cos p, 0)
 *    (Sec. 2.1); Q > 0 along theta_hat, U > 0 at +45 deg from theta_hat toward
 *    phi_hat, coherency rho = 1/2 [[I+Q, U-iV],[U+iV, I-Q]].
 *  - grid cell (i,j,k) covers [x0+i dx, x0+(i+1) dx) etc.; flat index
 *    c = i + nx*(j + ny*k); density and alignment arrays are float32.
 *  - Philox4x64-10, key = (seed, lambda index), counter of block b of packet p
 *    = (p, b, 0, 0); draw d uses word d%4 of block d/4;
 *    u = ((w >> 41) + 0.5) * 2^-23.
 */
#ifndef POLRAD_ORACLE_H
#define POLRAD_ORACLE_H
#include <stdint.h>
#include <stddef.h>
#ifdef __cplusplus
extern "C" {
#endif

/* Composite mesh with static refinement (reading M1): rx*ry*rz root blocks
 * of block^3 cells (x fastest), each the root of a tree of blocks; a block
 * is either a leaf holding block^3 cells or refined into its 8 octants
 * (octant bit 0: upper half in x, bit 1: y, bit 2: z), blocks of block^3
 * cells of half the size.  Nodes: the roots first (node r for root r), then
 * the children of each refined node as 8 consecutive nodes; child[i] is -1
 * for a leaf, else the index of its first child.  Leaves are numbered in
 * node order; cell k (x fastest) of leaf j has the flat index
 * j * block^3 + k.  max_level bounds the depth (0..20). */
typedef struct {
  int32_t rx, ry, rz, block, max_level;
  int32_t n_nodes;
  const int32_t *child;
} kpo_mesh;

typedef struct {
  int32_t nx, ny, nz;
  double x0, y0, z0, dx;        /* lower corner, cubic cell size */
  int32_t boundary;             /* bit a set: axis a (x, y, z) periodic, else open */
  const kpo_mesh *mesh;         /* NULL: the uniform grid nx*ny*nz; else the mesh,
                                   with nx = rx*block (likewise y, z) and dx the
                                   cell size of the root blocks; open boundaries */
} kpo_grid;

/* a packet ends as KPO_END_BUDGET after this many cell steps (a packet that
 * cannot scatter and moves parallel to every open face of a partly periodic
 * grid would never leave it) */
#define KPO_MAX_STEPS (1 << 24)

typedef struct {
  double kappa_sca, kappa_abs;  /* orientation-averaged, per unit rho per unit length */
  double a_perp_re, a_perp_im;  /* dipole polarizability across the symmetry axis */
  double a_par_re, a_par_im;    /* dipole polarizability along the symmetry axis  */
  double alpha3_scale;          /* artificial U-V extinction term: alpha3 = scale*alpha2 */
  /* tabulated scattering (reading T1), or n_theta = 0 for the dipole: the
   * scattering-plane matrix elements S11 S12 S22 S33 S34 S44 (any common
   * scale) at Theta_j = j pi / (n_theta - 1), j = 0..n_theta-1, linear in
   * cos Theta between nodes; the extinction is then scalar (the polarizabilities
   * are not used) */
  int32_t n_theta;
  const double *Z;              /* [n_theta][6] */
} kpo_dust;

typedef struct {
  int32_t kind;                 /* 0 isotropic point source, 1 pencil beam along dir,
                                   2 thermal emission of the dust (reading E1) */
  double pos[3], dir[3];
  double lum;                   /* luminosity per wavelength (kinds 0 and 1) */
  const float *B;               /* kind 2: source function of every cell [ncell]
                                   at this wavelength */
} kpo_source;

typedef struct {
  double theta, phi;            /* direction from the grid toward the observer (rad) */
  int32_t npx, npy;
  double half_width;            /* image spans [-W, W]^2 in the sky plane */
} kpo_view;

typedef struct {
  uint64_t seed;
  double rr_wmin;               /* roulette when I < rr_wmin * I0 (0 disables) */
  double rr_psurv;              /* survival probability */
  int64_t max_events;           /* scattering-event cap per packet */
  int32_t nthreads;             /* 0 = OpenMP default */
} kpo_opts;

enum { KPO_END_NONE = 0, KPO_EV_SCATTER = 1, KPO_END_ESCAPE = 2, KPO_EV_RR_SURVIVE = 3,
       KPO_END_RR_KILL = 4, KPO_END_BUDGET = 5, KPO_END_NUMERIC = 6 };

typedef struct {
  uint64_t packet;
  int32_t end_kind;
  int32_t events;               /* scattering events */
  int64_t steps;                /* cell steps (segments) */
  int64_t last_cell;            /* flat index of the last cell visited, -1 if none */
  double n[3];
  double stokes[4];
  uint64_t hash;                /* FNV-1a over (event kind, cell) of every event */
  double tau_path;              /* sum of |continuous extinction exponent| over segments */
} kpo_trace;

typedef struct {
  int64_t cell_steps, scatterings, trials, rr_kills, rr_survivals,
          escaped, budget, numeric;
  double e_emitted, e_escaped, e_absorbed, e_rr_killed, e_rr_gained, e_budget;
  double e_scat_delta;          /* sum of (I after - I before) over scatterings */
} kpo_stats;

/* Monte Carlo step (step 1 of two-step imaging) for packets [p_begin, p_end)
 * of one wavelength `lam` out of n_total packets (packet weight lum/n_total).
 * S (may be NULL): per-view scattering source, layout [cell][view][4] in the
 * camera basis of each view, accumulated (+=).  traces (may be NULL):
 * p_end-p_begin records.  stats accumulated (+=).  Returns 0 or a negative
 * error code. */
int kpo_transport(const kpo_grid *g, const float *rho, const float *bhat,
                  const kpo_dust *d, int32_t lam, const kpo_source *src,
                  int32_t n_views, const kpo_view *views,
                  uint64_t p_begin, uint64_t p_end, uint64_t n_total,
                  const kpo_opts *o, double *S, kpo_trace *traces,
                  kpo_stats *stats);

/* The same transport, imaging by peel-off (the direct Monte Carlo imaging
 * that Sec. 2.3 sets two-step imaging against): at every scattering event
 * the Stokes vector scattered toward each camera, attenuated along the line
 * of sight to the grid's edge, is added to the pixel the event projects to,
 * divided by the pixel's area.  peel: [view][4][npy][npx], accumulated.
 * Open boundaries only, on a uniform grid or a composite mesh; S may be
 * NULL. */
int kpo_transport_peel(const kpo_grid *g, const float *rho, const float *bhat,
                       const kpo_dust *d, int32_t lam, const kpo_source *src,
                       int32_t n_views, const kpo_view *views,
                       uint64_t p_begin, uint64_t p_end, uint64_t n_total,
                       const kpo_opts *o, double *S, double *peel, kpo_stats *stats);

/* Same transport for an explicit list of packet ids, traces only. */
int kpo_trace_packets(const kpo_grid *g, const float *rho, const float *bhat,
                      const kpo_dust *d, int32_t lam, const kpo_source *src,
                      const uint64_t *ids, uint64_t n_ids, uint64_t n_total,
                      const kpo_opts *o, kpo_trace *traces);

/* Step 2: deterministic ray-march of the source S ([cell][view][4]) toward
 * each camera.  images: [view][4][npy][npx] (all views must share npx, npy). */
int kpo_image(const kpo_grid *g, const float *rho, const float *bhat,
              const kpo_dust *d, int32_t n_views, const kpo_view *views,
              const double *S, double *images);
/* Step 2 with the dust's thermal emission added to the source (eq.
 * polarized-rt, alpha_abs B): B[ncell] the source function of every cell
 * (NULL: none); S may be NULL (no scattering source). */
int kpo_image_thermal(const kpo_grid *g, const float *rho, const float *bhat,
                      const kpo_dust *d, int32_t n_views, const kpo_view *views,
                      const double *S, const float *B, double *images);
/* Thermal emission draw of packet `packet` (reading E1): its cell, position
 * inside the cell (cell units), direction and Stokes vector (lab basis),
 * for a packet weight w. */
int kpo_emit_state(const kpo_grid *g, const float *rho, const float *bhat,
                   const kpo_dust *d, const float *B, uint64_t seed, int32_t lam,
                   uint64_t packet, double w, int64_t *cell, double pos[3], double n[3],
                   double s[4]);
/* Total thermal luminosity 4 pi sum_c rho_c kappa_abs B_c V of the grid. */
double kpo_emission_luminosity(const kpo_grid *g, const float *rho, const kpo_dust *d,
                               const float *B);

/* ---- building blocks, exported for the pin tests ---- */
void kpo_philox(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
double kpo_uniform(uint64_t seed, uint64_t lam, uint64_t packet, uint64_t draw);
void kpo_quat_from_b(const double b[3], double q[4]);
void kpo_to_grain(const double q[4], const double v[3], double out[3]);
void kpo_from_grain(const double q[4], const double v[3], double out[3]);
void kpo_basis(const double n[3], double th[3], double ph[3]);
double kpo_eta(const double q[4], const double n[3]);
void kpo_rotate_stokes(double eta, const double s[4], double out[4]);
void kpo_alphas(const kpo_dust *d, double cos_t, double a[3]);
void kpo_mueller_lab(const kpo_dust *d, const double q[4], const double m[3],
                     const double n[3], const double s[4], double out[4]);
void kpo_appA(double a1, double a2, double a3, double dtau,
              const double src[4], const double in[4], double out[4]);
void kpo_segment(double m1, double m2, double m3, double len,
                 const double in[4], double integral[4], double out[4]);
/* one scattering event drawn from the stream (seed, lam, packet) starting at
 * draw index first_draw; returns 0 or -1 (bound violated / no acceptance) */
int kpo_scatter_sample(const kpo_dust *d, const double q[4], const double n[3],
                       const double s[4], uint64_t seed, uint64_t lam, uint64_t packet,
                       uint64_t first_draw, double m_out[3], double s_out[4],
                       int64_t *trials);
double kpo_scatter_weight(const kpo_dust *d, const double q[4], const double n[3],
                          const double s[4]);

#ifdef __cplusplus
}
#endif
#endif
