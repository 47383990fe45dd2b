/*
 * polrad.h -- C ABI of the MI355X (gfx950) polarized Monte Carlo radiative
 * transfer library (libpolrad.so).
 *
 * The library implements the method of Yang & Wang, "Kratos-polrad: Novel GPU
 * system for Monte-Carlo simulations with consistent polarization
 * calculations" (arXiv:2512.01283): photon packets carrying the full Stokes
 * vector (I,Q,U,V) through a uniform Cartesian density grid (Sec. 2.2), with
 * per-cell analytic dichroic extinction (Appendix A), dipole Mueller-matrix
 * scattering in the grain frame reached by quaternions (Sec. 2.1), and
 * two-step imaging (Sec. 2.3): step 1 tallies the scattering source on the
 * grid from every path segment, step 2 ray-marches it to each camera.
 *
 * General rules
 *  - Every entry point returns kp_status; none throws or aborts.  On failure
 *    kp_last_error() gives a message.  Arguments are validated before any
 *    launch; an invalid argument leaves the context unchanged.
 *  - A context is bound to one HIP device and is not thread-safe; separate
 *    contexts are independent.
 *  - "host" pointers are ordinary CPU memory.  "device" pointers are HIP
 *    device allocations owned by the caller (borrowed: the caller keeps them
 *    alive and unchanged until the stream of the call that uses them has
 *    completed; the library never frees them).
 *  - hip_stream is a hipStream_t passed as void* (NULL = default stream).
 *  - Arrays over cells use the flat index c = i + nx*(j + ny*k), x fastest.
 *
 * Conventions (Sec. 2.1): a direction (theta, phi) has the Stokes basis
 * theta_hat = (cos t cos p, cos t sin p, -sin t), phi_hat = (-sin p, cos p, 0);
 * Q > 0 is polarisation along theta_hat, U > 0 at +45 degrees from theta_hat
 * toward phi_hat, V > 0 where the coherency is 1/2 [[I+Q, U-iV],[U+iV, I-Q]].
 */
#ifndef POLRAD_H
#define POLRAD_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KP_OK = 0,
  KP_ERR_ARG = 1,     /* invalid argument (nothing was launched) */
  KP_ERR_OOM = 2,     /* device memory exhausted or estimate exceeds free memory */
  KP_ERR_DEVICE = 3,  /* HIP runtime error */
  KP_ERR_STATE = 4,   /* call out of order (e.g. kp_run before kp_set_grid) */
  KP_ERR_NUMERIC = 5, /* a packet produced a non-finite state; results suspect */
  KP_ERR_BUDGET = 6   /* strict mode: a packet reached the scattering-event cap */
} kp_status;

typedef struct kp_ctx kp_ctx;

/* Uniform grid of cubic cells [x0 + i dx, x0 + (i+1) dx) x ... (Sec. 2.2).
 * boundary is a bit mask over the axes x, y, z (bit 0, 1, 2): a clear bit
 * makes both faces normal to that axis open (a packet crossing one escapes),
 * a set bit makes the axis periodic (a packet crossing one face re-enters
 * through the opposite one, and a camera ray runs on through the periodic
 * copies of the grid), the boundary condition of the Sec. 3.1 test.  0..6;
 * 7 (no open face) is rejected with KP_ERR_ARG.  With periodic axes a packet
 * ends after 2^24 cell steps (reported as a cap packet), and step 2 refuses
 * (KP_ERR_ARG) a camera whose rays would cross more than 2^24 cell lengths
 * before reaching an open face. */
typedef struct {
  int32_t nx, ny, nz;
  double x0, y0, z0, dx;
  int32_t boundary;
} kp_grid;

/* One dust species at one wavelength (Sec. 2.2, mfp-matrices equation):
 * kappa_sca, kappa_abs are orientation-averaged opacities per unit density per
 * unit length (lambda^-1 = rho * kappa).  The grain optics are a dipole
 * (Sec. 3): complex polarizabilities (re, im) across (a_perp) and along
 * (a_par) the grain symmetry axis, which is the local alignment direction;
 * only their ratios matter.  a_perp == a_par means spheres (Rayleigh).
 * alpha3_scale sets the artificial U-V extinction term alpha3 =
 * alpha3_scale * alpha2 used by the twisted-field verification (Sec. 3.2);
 * physical grains have 0. */
typedef struct {
  double kappa_sca, kappa_abs;
  double a_perp[2], a_par[2];
  double alpha3_scale;
} kp_dust;

/* kind 0: isotropic unpolarised point source at pos; kind 1: pencil beam from
 * pos along dir (tests).  lum is the luminosity per wavelength; each packet
 * of a wavelength with N packets starts with I = lum / N.  pos must lie in
 * the closed grid box.
 * kind 2: thermal emission of the dust (Sec. 2.2, the alpha_abs B term of
 * eq. polarized-rt) with the source function set by kp_set_emission; pos,
 * dir and lum are ignored.  A cell's luminosity is 4 pi rho kappa_abs B dx^3
 * and L the sum over cells; packets start in a cell drawn in proportion to
 * it, uniformly inside the cell, in an isotropic direction, with the Stokes
 * vector (L / N) (alpha1, alpha2, 0, 0) in the grain-frame basis of that
 * direction: the absorption matrix is taken as kappa_abs / kappa_ext times
 * the extinction matrix (Appendix A with the source (alpha1, alpha2) B when
 * all extinction is absorption); its mean over directions is L / N.  Step 2
 * then adds (kappa_abs / kappa_ext)(alpha1, alpha2, 0, 0) B per unit optical
 * depth to the scattering source. */
typedef struct {
  int32_t kind;
  double pos[3], dir[3];
  double lum;
} kp_source;

/* Camera (Sec. 2.3): direction (theta, phi) from the grid toward the
 * observer; orthographic, npx x npy pixels spanning [-half_width, half_width]^2
 * in the sky plane through the origin, image x along phi_hat, image y along
 * -theta_hat; Stokes in the (theta_hat, phi_hat) basis of the camera
 * direction.  All views of a context share npx and npy. */
typedef struct {
  double theta, phi;
  int32_t npx, npy;
  double half_width;
} kp_view;

/* Run options.
 *  seed            Philox4x64-10 key word 0 (key word 1 = wavelength index).
 *  transport_fp64  arithmetic of step 1 (tallies are FP64 in every mode):
 *                  0 = automatic: FP32 polarisation arithmetic for spherical
 *                      grains, FP64 for aligned non-spherical grains;
 *                  1 = FP64 throughout (parity runs);
 *                  2 = FP32 polarisation arithmetic for every grain type.
 *                  Geometry (positions, directions, scattering depths) is
 *                  FP64 in every mode.  Aligned grains default to FP64
 *                  because a thick dichroic cell (App. A) scales the two
 *                  grain-frame components I+Q and I-Q by e^{-x_A} and e^{-x_B}
 *                  with |x_A - x_B| up to ~10: it amplifies the ~6e-8 I
 *                  representation error of an FP32 Stokes vector in the
 *                  small component by up to e^{|x_A - x_B|}, so a few packets
 *                  per thousand end with relative errors of 1e-4..1e-3.
 *  tally_mode      0 (only value): per-cell incident coherency tally.
 *  rr_wmin, rr_psurv  Russian roulette when I < rr_wmin * I0 (0 disables).
 *  max_events      scattering-event cap per packet (>= 1).
 *  trace_packets   number of packets per wavelength whose final state is
 *                  recorded (ids 0, trace_stride, 2 trace_stride, ...).
 *  trace_stride    >= 1.
 *  block_size      threads per block of the transport kernel (64, 128, 192
 *                  or 256; 0 = default 256; KP_ERR_ARG otherwise).
 *  blocks_per_cu   resident blocks per compute unit (0 = default).
 *  strict          1: kp_run returns KP_ERR_BUDGET if any packet hit the cap.
 *  scatter_batch   a lane that reaches a scattering point waits until this
 *                  many lanes of its wavefront do (1..64; 0 = default 8) ...
 *  scatter_wait    ... or until it has waited this many iterations (1..1024;
 *                  0 = default 16).  Scheduling only: results are identical
 *                  for every setting (each packet keeps its own streams).
 *  peel_off        1: also form peel-off images (the direct Monte Carlo
 *                  imaging that Sec. 2.3 sets two-step imaging against): at
 *                  every scattering event, for every camera, the Stokes
 *                  vector scattered toward the camera per unit solid angle
 *                  (from the packet's own incident coherency, as step 2
 *                  forms its source from the tallied one), attenuated
 *                  through every cell to the grid's edge with the Appendix A
 *                  extinction, per unit pixel area, in the pixel the event
 *                  projects to.  Scattered light only (no direct light of
 *                  the source or the dust).  Read with kp_get_peel_images.
 *                  Needs open boundaries (boundary 0) and kp_run or
 *                  kp_transport (KP_ERR_ARG otherwise).  0 = off.
 * block_size, blocks_per_cu, scatter_batch and scatter_wait are what the
 * autotuner searches. */
typedef struct {
  uint64_t seed;
  int32_t transport_fp64;
  int32_t tally_mode;
  double rr_wmin, rr_psurv;
  int64_t max_events;
  uint32_t trace_packets;
  uint32_t trace_stride;
  int32_t block_size;
  int32_t blocks_per_cu;
  int32_t strict;
  int32_t scatter_batch;
  int32_t scatter_wait;
  int32_t peel_off;
} kp_opts;

/* Counters of the last kp_run/kp_transport (energies in units of lum). */
typedef struct {
  int64_t cell_steps, scatterings, trials, rr_kills, rr_survivals,
          escaped, budget, numeric;
  double e_emitted, e_escaped, e_absorbed, e_rr_killed, e_rr_gained, e_budget,
         e_scat_delta;
  double ms_transport; /* transport kernel time (HIP events on the run's stream) */
  double ms_image;     /* imaging kernel time */
  int64_t packets;
  int64_t tally_flushes; /* per-cell tally blocks added to the source tally
                            (one atomic read-modify-write of the block each) */
} kp_stats;

/* Final state of a traced packet. end_kind: 2 escaped, 4 roulette kill or
 * absorbed, 5 event cap, 6 non-finite state.  hash: FNV-1a-64 over the
 * 4-byte little-endian (kind, cell) pairs of its events (1 scatter,
 * 2 escape, 3 roulette survival, 4 roulette kill, 5 cap).  tau_path: sum
 * over its segments of the magnitude of the continuous-extinction exponent
 * (rho kappa_ext alpha1 - rho kappa_sca) * length. */
typedef struct {
  uint64_t packet;
  int32_t end_kind;
  int32_t events;
  int64_t steps;
  int64_t last_cell;
  double n[3];
  double stokes[4];
  uint64_t hash;
  double tau_path;
} kp_packet_trace;

/* Create a context on HIP device `device`: the device state of one problem
 * of the method (Sec. 2.2 grid, dust and source; Sec. 2.3 cameras).  *out
 * receives an owned handle (release with kp_destroy).  KP_ERR_DEVICE if no
 * HIP device is present, KP_ERR_ARG for a device index out of range. */
kp_status kp_create(int device, kp_ctx **out);
/* Release a context and every device buffer it owns (Sec. 2.2-2.3 state);
 * borrowed device arrays are not freed.  NULL is ignored. */
void kp_destroy(kp_ctx *ctx);
/* Message of the last failed call on ctx (owned by the context, valid until
 * its next call); covers every entry point of the Sec. 2.2-2.3 method. */
const char *kp_last_error(const kp_ctx *ctx);

/* The medium (Sec. 2.2: density profile read in as the input of the
 * opacities, eq. mfp-matrices; Sec. 2.1: the grain alignment direction that
 * defines the grain frame, eq. grain-quaternion).  Density rho[ncell]
 * (float32, finite, >= 0) and optional unit alignment field bhat[3][ncell]
 * (float32 SoA, |b| = 1 within 1e-5; NULL = no alignment: the grain frame
 * coincides with the lab frame).  kp_set_grid copies host arrays into
 * library-owned device memory; kp_set_grid_device borrows device arrays
 * (validated by a device pass: KP_ERR_ARG with the count of bad values).
 * Either resets the tally. */
kp_status kp_set_grid(kp_ctx *ctx, const kp_grid *grid, const float *rho, const float *bhat);
kp_status kp_set_grid_device(kp_ctx *ctx, const kp_grid *grid, const float *d_rho,
                             const float *d_bhat);

/* Composite mesh with static refinement (Sec. 2: the mesh grid the packets
 * cross, optionally statically refined).  rx*ry*rz root blocks (x fastest)
 * of block^3 cubic cells of edge dx tile the box from (x0, y0, z0); each
 * block is a leaf or is refined into its 8 octants (octant bit 0: the upper
 * half in x, bit 1: y, bit 2: z), blocks of block^3 cells of half the edge,
 * to at most max_level refinements.  child[n_nodes] lists the blocks: the
 * roots first (node r for root block r), then the 8 children of each
 * refined node as 8 consecutive nodes after it; child[i] is -1 for a leaf,
 * else the index of its first child.  Leaves are numbered in node order and
 * cell k (x fastest) of leaf j is cell j*block^3 + k of every per-cell
 * array: rho[ncell] (float32, finite, >= 0) and the optional alignment
 * field bhat[3][ncell] as in kp_set_grid, ncell = leaves * block^3.  A
 * packet or camera ray crosses a leaf's cells as on a uniform grid; leaving
 * the block it continues in the leaf holding the exit point (a coordinate
 * on a face belongs to the cell the direction points into); every cell's
 * length, volume and thermal luminosity are those of its level.  Open
 * boundaries.  1 <= block <= 64, 0 <= max_level <= 16, the box at most 2^30
 * finest cells along each axis, ncell <= 4e9; KP_ERR_ARG for a malformed
 * tree (a node with two parents or none, children before their parent or
 * past the list, depth beyond max_level).  Copies the arrays to the
 * device; replaces any grid (kp_set_grid replaces the mesh) and resets the
 * tally. */
typedef struct {
  int32_t rx, ry, rz;
  int32_t block;
  int32_t max_level;
  int32_t n_nodes;
  double x0, y0, z0, dx;
} kp_mesh;
kp_status kp_set_mesh(kp_ctx *ctx, const kp_mesh *mesh, const int32_t *child, const float *rho,
                      const float *bhat);

/* Grain optics per wavelength (Sec. 2.2, eq. mfp-matrices and the
 * user-defined cross sections and Mueller matrices; Sec. 3 dipole grains):
 * n_lambda (1..1024) dust records, one per wavelength (copied).  KP_ERR_ARG
 * for negative or non-finite opacities or polarizabilities. */
kp_status kp_set_dust(kp_ctx *ctx, int32_t n_lambda, const kp_dust *dust);
/* Tabulated scattering for every wavelength (Sec. 2.2: the differential
 * cross section and Mueller matrix given by the user as interpolation
 * tables).  Z[n_lambda][n_theta][6] (host, FP64, copied) holds the
 * scattering-plane elements S11 S12 S22 S33 S34 S44 of randomly oriented
 * grains (or spheres) at the scattering angles Theta_j = j pi / (n_theta-1),
 * in any common scale per wavelength; the matrix is
 * [[S11,S12,0,0],[S12,S22,0,0],[0,0,S33,S34],[0,0,-S34,S44]] with Q along the
 * scattering plane (Bohren & Huffman), V as in this header's Stokes
 * convention (S34 = Im(S2 conj(S1)) for amplitude functions S2 parallel, S1
 * perpendicular), linear in cos Theta between nodes, normalised by the
 * library to unit solid-angle integral of S11.  With tables the extinction
 * is scalar (kappa_sca + kappa_abs of kp_dust; the polarizabilities are not
 * used and alignment directions are ignored), scattering directions are
 * drawn from the table, and step 1 tallies the per-view source of Sec. 2.3
 * (eq. scat-disc-sum: one Stokes vector per cell and camera, [n_lambda]
 * [ncell][n_views][4] FP64, read with kp_get_view_tally) instead of the
 * coherency, which is exact only for dipoles; kp_set_views then invalidates
 * the tally.  n_lambda must equal kp_set_dust's (called first; kp_set_dust
 * discards the tables); 2 <= n_theta <= 65536; every |S_ij| <= S11 at every
 * node, finite, with a positive integral (KP_ERR_ARG otherwise).
 * n_lambda = 0 with Z = NULL returns to dipole grains. */
kp_status kp_set_dust_tables(kp_ctx *ctx, int32_t n_lambda, int32_t n_theta, const double *Z);
/* The radiation source whose packets are emitted (Sec. 2.2: packets are
 * generated and given an exponentially distributed scattering optical
 * depth); copied.  KP_ERR_ARG for an unknown kind, a non-positive
 * luminosity or a zero pencil direction (kinds 0 and 1). */
kp_status kp_set_source(kp_ctx *ctx, const kp_source *src);
/* Source function of the dust's thermal emission (Sec. 2.2, B of eq.
 * polarized-rt; used by source kind 2): B[n_lambda][ncell] (host, float32,
 * finite, >= 0), e.g. the Planck function of each cell's temperature at each
 * wavelength, in the units the images are wanted in (lengths in the grid's
 * unit); copied to the device.  n_lambda must equal kp_set_dust's at the
 * next run.  Needs a grid; kp_set_grid / kp_set_grid_device discard it.
 * KP_ERR_ARG for a negative or non-finite value. */
kp_status kp_set_emission(kp_ctx *ctx, int32_t n_lambda, const float *B);
/* Cameras of step 2 (Sec. 2.3, the camera direction Omega_cam of eq.
 * scat-disc-sum): n_views (1..4096) views (copied), all with the same npx,
 * npy (1..16384). */
kp_status kp_set_views(kp_ctx *ctx, int32_t n_views, const kp_view *views);

/* Two-step imaging (Sec. 2.3): step 1 (packet transport, Sec. 2.2 and
 * Appendix A, tallying the scattering source of eq. scat-disc-sum) + step 2
 * (ray-march to every camera) for all wavelengths, in one persistent launch
 * each: packets_per_lambda[n_lambda] (host, >= 0, total >= 1).  Images stay
 * on the device; the call synchronises hip_stream before returning (it
 * reads the counters back).  Returns KP_ERR_NUMERIC / KP_ERR_BUDGET (strict)
 * after a completed run whose counters show them. */
kp_status kp_run(kp_ctx *ctx, const uint64_t *packets_per_lambda, const kp_opts *opts,
                 void *hip_stream);
/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): kp_run
 * without any allocation.  Step 1 and step 2 run as in kp_run, with the
 * counters, the per-wavelength and camera tables and the step-1 tally held
 * in one static device array of the library (1 MiB + 256 MiB, one copy per
 * device, held until the process ends) instead of context buffers; the
 * images go straight to d_images (device, borrowed, [n_lambda][n_views][4]
 * [npy][npx] FP64, n its element count).  Limits: the tally, n_lambda x
 * nslot x 64 B for spherical grains (x 128 B for aligned grains, x 32 B x
 * n_views for tabulated ones), with nslot = ncell on a composite mesh and
 * 64 ceil(nx/4) ceil(ny/4) ceil(nz/4) on a uniform grid (whose tally keeps
 * its cells in bricks of 4 x 4 x 4), must fit 256 MiB (KP_ERR_ARG
 * otherwise, before any launch: use kp_run), and no traces are
 * recorded (trace_packets must be 0) and no peel-off images formed
 * (peel_off must be 0).  kp_get_stats then reports this call;
 * kp_image, kp_get_images and kp_get_tally keep referring to the last
 * kp_run / kp_transport.  Every call on one device uses that device's one
 * array, cleared at the start of each call by kernels: calls that overlap
 * on one device (two streams, threads or contexts) race and must not be
 * issued.  Synchronises hip_stream. */
kp_status kp_run_static(kp_ctx *ctx, const uint64_t *packets_per_lambda, const kp_opts *opts,
                        double *d_images, size_t n, void *hip_stream);
/* Step 1 only (Sec. 2.3 first step, transport of Sec. 2.2 with the
 * Appendix A cell solution): tallies the scattering source of eq.
 * scat-disc-sum as each cell's incident coherency.  Same arguments, errors
 * and synchronisation as kp_run. */
kp_status kp_transport(kp_ctx *ctx, const uint64_t *packets_per_lambda, const kp_opts *opts,
                       void *hip_stream);
/* Step 2 only (Sec. 2.3 second step: eq. polarized-rt integrated along each
 * line of sight with the Appendix A cell solution), from the tally of the
 * last kp_transport; synchronises hip_stream.  KP_ERR_STATE without a
 * tally. */
kp_status kp_image(kp_ctx *ctx, void *hip_stream);
/* Step 2 alone (Sec. 2.3 second step, Appendix A with the source S) on a
 * caller-supplied per-view source of eq. scat-disc-sum (wavelength 0):
 * d_S device [ncell][n_views][4] FP64, emissivity per unit length per unit
 * solid angle in each camera basis; d_out device [n_views][4][npy][npx]
 * (both borrowed).  Synchronises hip_stream. */
kp_status kp_image_source(kp_ctx *ctx, const double *d_S, double *d_out, void *hip_stream);

/* Stokes images of the last step 2 (Sec. 2.3: the synthetic polarimetry
 * maps), [n_lambda][n_views][4][npy][npx] FP64; n is the element count of
 * the destination and must equal that size (KP_ERR_ARG otherwise,
 * KP_ERR_STATE before any step 2).  kp_get_images copies to host memory and
 * synchronises; kp_get_images_device copies on hip_stream into a borrowed
 * device array. */
kp_status kp_get_images(kp_ctx *ctx, double *host_out, size_t n);
kp_status kp_get_images_device(kp_ctx *ctx, double *d_out, size_t n, void *hip_stream);
/* Peel-off images of the last step 1 run with opts.peel_off = 1 (the
 * Monte Carlo imaging Sec. 2.3 compares two-step imaging with; kp_opts
 * above), same layout and units as kp_get_images: [n_lambda][n_views][4]
 * [npy][npx] FP64, copied to host memory; n must equal that size
 * (KP_ERR_ARG otherwise, KP_ERR_STATE if the last step 1 formed none). */
kp_status kp_get_peel_images(kp_ctx *ctx, double *host_out, size_t n);
/* Incident-coherency tally [n_lambda][ncell][9] FP64 of the last step 1
 * (the scattering source of Sec. 2.3, eq. scat-disc-sum, before the camera
 * projection: components xx yy zz xy xz yz and the imaginary yz zx xy
 * parts), per unit cell volume times dx^3, cells in the order of the
 * density array whatever layout the device keeps them in; n must equal
 * that size. */
kp_status kp_get_tally(kp_ctx *ctx, double *host_out, size_t n);
/* Per-view scattering source of the last step 1 with tabulated grains (Sec.
 * 2.3, eq. scat-disc-sum: the emissivity toward each camera per unit volume
 * and solid angle, in that camera's basis), [n_lambda][ncell][n_views][4]
 * FP64, cells in the order of the density array, copied to host memory;
 * n must equal that size (KP_ERR_ARG), and
 * KP_ERR_STATE when the last step 1 tallied coherencies (dipole grains,
 * kp_get_tally) or formed none. */
kp_status kp_get_view_tally(kp_ctx *ctx, double *host_out, size_t n);
/* Counters of the last step 1 and step 2 (Sec. 2.2 packet events; kp_stats
 * above), copied to *out. */
kp_status kp_get_stats(kp_ctx *ctx, kp_stats *out);
/* Final states of the traced packets of the last step 1 (Sec. 2.2 packet
 * histories; kp_packet_trace above): n must equal n_lambda * trace_packets. */
kp_status kp_get_trace(kp_ctx *ctx, kp_packet_trace *out, size_t n);

#ifdef __cplusplus
}
#endif
#endif
