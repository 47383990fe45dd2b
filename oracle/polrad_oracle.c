/*
 * polrad_oracle.c -- FP64 CPU oracle for polarized Monte Carlo radiative
 * transfer with two-step imaging, after Yang & Wang, "Kratos-polrad: Novel GPU
 * system for Monte-Carlo simulations with consistent polarization
 * calculations" (arXiv:2512.01283).
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow, step-by-step statement of what the
 * method computes.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never does.  It shares
 * no code with the HIP library.
 *
 * Every routine names the passage of the paper it follows.  Where the paper is
 * silent or its printed formula is inconsistent, the reading taken is stated
 * at the routine (the same readings are listed in the design notes):
 *  R1 extinction matrix signs (Appendix A): the printed solution is the
 *     reference; it fixes K = [[a1,a2,0,0],[a2,a1,0,0],[0,0,a1,a3],[0,0,-a3,a1]].
 *  R2 sign of eta (Sec. 2.1, rotation-angle equation): signed,
 *     sin(eta) = n_GF . (phi_GF x phi'), cos(eta) = phi_GF . phi'.
 *  R3 optical depth sampled (Sec. 2.2): exponential in the scattering optical
 *     depth with rate kbar = rho*kappa_sca; the rest of the extinction acts on
 *     the Stokes vector continuously as exp(-(K - kbar) l).
 *  R4 grain optics (Sec. 3 intro, dipole approximation): polarizability
 *     diag(a_perp, a_perp, a_par) in the grain frame; extinction from Im
 *     (optical theorem), normalised by the orientation average.
 *  R5 segment contribution to S (Sec. 2.3): the exact integral of the Stokes
 *     vector over the segment, times rho*kappa_sca / V_cell, through the
 *     Mueller matrix normalised to unit solid-angle integral.
 *  R6 rejection sampling (Sec. 3 intro): proposals uniform on the sphere in
 *     the grain frame, bound 3/(8 pi N_P) max(|a_perp|^2,|a_par|^2) I.
 *  R7 weight after scattering: I' = tr(alpha C alpha^dagger)/N_P.
 *  R8 termination: escape through an open face, Russian roulette, event
 *     cap, and a cap of KPO_MAX_STEPS cell steps.
 *  R14 boundaries (Sec. 3.1 uses periodic ones): each axis open or periodic;
 *     a packet crossing a periodic face re-enters through the opposite one,
 *     and a camera ray runs through the periodic copies of the grid from the
 *     open face where it enters to the open face where it leaves.
 *  R9 orthographic camera, image x along phi_hat, y along -theta_hat.
 *  T1 tabulated optical properties (Sec. 2.2: user-defined interpolation
 *     tables): a medium of randomly oriented grains with mirror symmetry
 *     (or spheres), whose scattering-plane Mueller matrix has the block form
 *     [[S11,S12,0,0],[S12,S22,0,0],[0,0,S33,S34],[0,0,-S34,S44]] of the
 *     scattering angle only (Bohren & Huffman's convention: Q along the
 *     scattering plane, here with V as in R10, so S34 = Im(S2 conj(S1)) for
 *     amplitude functions S2 (parallel) and S1 (perpendicular)); tabulated at
 *     Theta uniform on [0, pi], linear in cos Theta between nodes, normalised
 *     so that the solid-angle integral of S11 is 1; scalar extinction.
 *  T2 sampling of a tabulated scattering (Sec. 2.2): envelope rejection,
 *     the envelope on each node interval the larger S11 of its two nodes
 *     times (I + sqrt(Q^2+U^2)); draws per trial: interval (by the envelope's
 *     cumulative mass), cos Theta uniform in the interval, azimuth, accept.
 *  M1 static mesh refinement (Sec. 2: a composite mesh, optionally with
 *     static refinement): root blocks of block^3 cells on a uniform array,
 *     each refinable into its 8 octants recursively (see kpo_mesh); packets
 *     and camera rays cross cells of a leaf block as on a uniform grid and,
 *     leaving it, continue in the leaf holding the exit point, found in
 *     units of the finest cell with the face rule of R12.  Cell lengths and
 *     volumes are those of the cell's level (a cell's thermal luminosity
 *     4 pi rho kappa_abs B V with its own V).  Open boundaries.
 *  E1 thermal emission of the dust (Sec. 2.2, the alpha_abs B term of eq.
 *     polarized-rt): the absorption matrix is kappa_abs/kappa_ext times the
 *     extinction matrix, so a cell emits rho kappa_abs (alpha1, alpha2, 0, 0) B
 *     per unit length and solid angle in the grain-frame basis of the
 *     direction (the source (alpha1, alpha2) B of Appendix A when all
 *     extinction is absorption); its orientation average is rho kappa_abs B,
 *     so a cell's luminosity is 4 pi rho kappa_abs B V.
 */
#include "polrad_oracle.h"
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI_ 3.14159265358979323846264338327950288
#define POLE_EPS2 8.673617379884035e-19 /* 2^-60 */

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two     */
/* 64x64->128 multiplies with a Weyl-sequence key schedule.                  */
/* ------------------------------------------------------------------------ */
void kpo_philox(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    unsigned __int128 p0 = (unsigned __int128)M0 * x0;
    unsigned __int128 p1 = (unsigned __int128)M1 * x2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    x0 = hi1 ^ x1 ^ k0;
    x1 = lo1;
    x2 = hi0 ^ x3 ^ k1;
    x3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

typedef struct {
  uint64_t key[2];
  uint64_t packet;
  uint64_t next;     /* next draw index */
  uint64_t block;    /* block held in buf */
  int have;
  uint64_t buf[4];
} rng_t;

static double word_to_uniform(uint64_t w) {
  /* 23 high bits, centred: (k + 1/2) 2^-23, strictly inside (0,1) and exact in
   * both float32 and float64 */
  return ((double)(w >> 41) + 0.5) * (1.0 / 8388608.0);
}

static double draw(rng_t *r) {
  uint64_t d = r->next++;
  uint64_t b = d >> 2;
  if (!r->have || r->block != b) {
    uint64_t c[4] = {r->packet, b, 0, 0};
    kpo_philox(c, r->key, r->buf);
    r->block = b;
    r->have = 1;
  }
  return word_to_uniform(r->buf[d & 3]);
}

double kpo_uniform(uint64_t seed, uint64_t lam, uint64_t packet, uint64_t drawi) {
  rng_t r = {{seed, lam}, packet, drawi, 0, 0, {0, 0, 0, 0}};
  return draw(&r);
}

/* ------------------------------------------------------------------------ */
/* small vector helpers                                                      */
/* ------------------------------------------------------------------------ */
static double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(const double a[3], const double b[3], double o[3]) {
  double t0 = a[1] * b[2] - a[2] * b[1];
  double t1 = a[2] * b[0] - a[0] * b[2];
  double t2 = a[0] * b[1] - a[1] * b[0];
  o[0] = t0; o[1] = t1; o[2] = t2;
}

/* ------------------------------------------------------------------------ */
/* Quaternions (Sec. 2.1).  q = (q0, q1, q2, q3) = q0 + q1 i + q2 j + q3 k.  */
/* ------------------------------------------------------------------------ */
static void qmul(const double a[4], const double b[4], double o[4]) {
  double w = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  double x = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
  double y = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
  double z = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
  o[0] = w; o[1] = x; o[2] = y; o[3] = z;
}

/* Grain-frame quaternion from the alignment direction (theta_B, phi_B),
 * grain-quaternion equation of Sec. 2.1. */
void kpo_quat_from_b(const double b_in[3], double q[4]) {
  double nb = sqrt(dot3(b_in, b_in));
  double b[3] = {b_in[0] / nb, b_in[1] / nb, b_in[2] / nb};
  double rxy2 = b[0] * b[0] + b[1] * b[1];
  double thB = atan2(sqrt(rxy2), b[2]);
  double phB = rxy2 <= POLE_EPS2 ? 0.0 : atan2(b[1], b[0]);
  q[0] = cos(0.5 * phB) * cos(0.5 * thB);
  q[1] = -sin(0.5 * phB) * sin(0.5 * thB);
  q[2] = cos(0.5 * phB) * sin(0.5 * thB);
  q[3] = sin(0.5 * phB) * cos(0.5 * thB);
}

/* (0, v_GF) = q^* (0, v) q   (vector-transform equation, Sec. 2.1) */
void kpo_to_grain(const double q[4], const double v[3], double out[3]) {
  double qc[4] = {q[0], -q[1], -q[2], -q[3]};
  double pv[4] = {0.0, v[0], v[1], v[2]};
  double t[4], r[4];
  qmul(qc, pv, t);
  qmul(t, q, r);
  out[0] = r[1]; out[1] = r[2]; out[2] = r[3];
}

/* inverse map: (0, v) = q (0, v_GF) q^* */
void kpo_from_grain(const double q[4], const double v[3], double out[3]) {
  double qc[4] = {q[0], -q[1], -q[2], -q[3]};
  double pv[4] = {0.0, v[0], v[1], v[2]};
  double t[4], r[4];
  qmul(q, pv, t);
  qmul(t, qc, r);
  out[0] = r[1]; out[1] = r[2]; out[2] = r[3];
}

/* Stokes reference basis of a direction (Sec. 2.1).  At the poles
 * (nx^2+ny^2 <= 2^-60) phi is taken as 0. */
void kpo_basis(const double n[3], double th[3], double ph[3]) {
  double rxy2 = n[0] * n[0] + n[1] * n[1];
  double t = atan2(sqrt(rxy2), n[2]);
  double p = rxy2 <= POLE_EPS2 ? 0.0 : atan2(n[1], n[0]);
  th[0] = cos(t) * cos(p);
  th[1] = cos(t) * sin(p);
  th[2] = -sin(t);
  ph[0] = -sin(p);
  ph[1] = cos(p);
  ph[2] = 0.0;
}

/* Signed angle between the lab phi_hat carried into the grain frame and the
 * natural phi_hat' of the grain-frame direction (rotation-angle equation,
 * reading R2).  v is the lab direction, vg its grain-frame image. */
static double eta_pair(const double q[4], const double v[3], const double vg[3]) {
  double th[3], ph[3], thg[3], phg[3], ph_in_g[3], cr[3];
  kpo_basis(v, th, ph);
  kpo_to_grain(q, ph, ph_in_g);
  kpo_basis(vg, thg, phg);
  cross3(ph_in_g, phg, cr);
  double s = dot3(vg, cr);
  double c = dot3(ph_in_g, phg);
  return atan2(s, c);
}

double kpo_eta(const double q[4], const double n[3]) {
  double ng[3];
  kpo_to_grain(q, n, ng);
  return eta_pair(q, n, ng);
}

/* Stokes rotation (stokes-rotation equation, Sec. 2.1): I and V invariant. */
void kpo_rotate_stokes(double eta, const double s[4], double out[4]) {
  double c2 = cos(2.0 * eta), s2 = sin(2.0 * eta);
  double Q = c2 * s[1] + s2 * s[2];
  double U = -s2 * s[1] + c2 * s[2];
  out[0] = s[0]; out[1] = Q; out[2] = U; out[3] = s[3];
}

/* ------------------------------------------------------------------------ */
/* Dipole grain optics (reading R4).                                         */
/* ------------------------------------------------------------------------ */
static int is_table(const kpo_dust *d) { return d->n_theta >= 2 && d->Z != NULL; }

static int is_sphere(const kpo_dust *d) {
  return is_table(d) || (d->a_perp_re == d->a_par_re && d->a_perp_im == d->a_par_im);
}

/* Dimensionless extinction coefficients alpha_1..3 of the transfer equation
 * (Sec. 2.2, Appendix A) for a direction at polar angle t' from the grain
 * axis.  C_theta/C_phi are the cross sections for E along theta'/phi'. */
void kpo_alphas(const kpo_dust *d, double cos_t, double a[3]) {
  if (is_sphere(d)) { a[0] = 1.0; a[1] = 0.0; a[2] = 0.0; return; }
  double sin2 = 1.0 - cos_t * cos_t;
  double c_th = d->a_perp_im * cos_t * cos_t + d->a_par_im * sin2;
  double c_ph = d->a_perp_im;
  double c_avg = (2.0 * d->a_perp_im + d->a_par_im) / 3.0;
  a[0] = (c_th + c_ph) / (2.0 * c_avg);
  a[1] = (c_th - c_ph) / (2.0 * c_avg);
  a[2] = d->alpha3_scale * a[1];
}

static double norm_p(const kpo_dust *d) {
  double ap2 = d->a_perp_re * d->a_perp_re + d->a_perp_im * d->a_perp_im;
  double aa2 = d->a_par_re * d->a_par_re + d->a_par_im * d->a_par_im;
  return (2.0 * ap2 + aa2) / 3.0;
}

/* Scattering Mueller matrix applied in the grain frame (Sec. 2.2, dipole
 * approximation of Sec. 3): Jones J_ij = f_i . alpha . e_j between the
 * natural bases of the incident (ng) and scattered (mg) grain-frame
 * directions; rho_out = J rho_in J^dagger; normalised so the solid-angle
 * integral of the scattered I is 1 for unpolarised light on
 * orientation-averaged grains (reading R5). */
static void mueller_grain(const kpo_dust *d, const double mg[3], const double ng[3],
                          const double s[4], double out[4]) {
  double e[2][3], f[2][3];
  kpo_basis(ng, e[0], e[1]);
  kpo_basis(mg, f[0], f[1]);
  double complex a[3] = {d->a_perp_re + I * d->a_perp_im, d->a_perp_re + I * d->a_perp_im,
                         d->a_par_re + I * d->a_par_im};
  double complex J[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      J[i][j] = 0.0;
      for (int k = 0; k < 3; ++k) J[i][j] += f[i][k] * a[k] * e[j][k];
    }
  double complex rho[2][2] = {{0.5 * (s[0] + s[1]), 0.5 * (s[2] - I * s[3])},
                              {0.5 * (s[2] + I * s[3]), 0.5 * (s[0] - s[1])}};
  double complex t[2][2], ro[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) t[i][j] = J[i][0] * rho[0][j] + J[i][1] * rho[1][j];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) ro[i][j] = t[i][0] * conj(J[j][0]) + t[i][1] * conj(J[j][1]);
  double k = 3.0 / (8.0 * PI_ * norm_p(d));
  out[0] = k * creal(ro[0][0] + ro[1][1]);
  out[1] = k * creal(ro[0][0] - ro[1][1]);
  out[2] = k * 2.0 * creal(ro[0][1]);
  out[3] = -k * 2.0 * cimag(ro[0][1]);
}

/* P(m; n) s with both Stokes vectors in lab bases: into the grain frame by
 * quaternion + eta rotation, Mueller there, and back (Sec. 2.1-2.2). */
static double table_norm(const kpo_dust *d);
static void table_mueller_lab(const kpo_dust *d, double N, const double m[3], const double n[3],
                              const double s[4], double out[4]);

void kpo_mueller_lab(const kpo_dust *d, const double q[4], const double m[3],
                     const double n[3], const double s[4], double out[4]) {
  if (is_table(d)) { table_mueller_lab(d, table_norm(d), m, n, s, out); return; }
  double ng[3], mg[3], sg[4], og[4];
  kpo_to_grain(q, n, ng);
  kpo_to_grain(q, m, mg);
  kpo_rotate_stokes(eta_pair(q, n, ng), s, sg);
  mueller_grain(d, mg, ng, sg, og);
  kpo_rotate_stokes(-eta_pair(q, m, mg), og, out);
}

/* tr(alpha C alpha^dagger)/N_P, C = sum_ab rho_ab e_a e_b^T the incident 3x3
 * coherency (reading R7), Stokes s in the grain-frame natural basis of ng. */
static double scatter_weight_grain(const kpo_dust *d, const double ng[3], const double s[4]) {
  double e[2][3];
  kpo_basis(ng, e[0], e[1]);
  double complex rho[2][2] = {{0.5 * (s[0] + s[1]), 0.5 * (s[2] - I * s[3])},
                              {0.5 * (s[2] + I * s[3]), 0.5 * (s[0] - s[1])}};
  double complex C[3][3];
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) {
      C[k][l] = 0.0;
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) C[k][l] += rho[a][b] * e[a][k] * e[b][l];
    }
  double complex al[3] = {d->a_perp_re + I * d->a_perp_im, d->a_perp_re + I * d->a_perp_im,
                          d->a_par_re + I * d->a_par_im};
  double tr = 0.0;
  for (int k = 0; k < 3; ++k) tr += creal(al[k] * C[k][k] * conj(al[k]));
  return tr / norm_p(d);
}

double kpo_scatter_weight(const kpo_dust *d, const double q[4], const double n[3],
                          const double s[4]) {
  if (is_table(d)) return s[0];  /* T1: the scattered power does not depend on polarisation */
  double ng[3], sg[4];
  kpo_to_grain(q, n, ng);
  kpo_rotate_stokes(eta_pair(q, n, ng), s, sg);
  return scatter_weight_grain(d, ng, sg);
}

/* ------------------------------------------------------------------------ */
/* Tabulated scattering matrices (Sec. 2.2: optical properties given as      */
/* interpolation tables; readings T1, T2).                                   */
/* ------------------------------------------------------------------------ */
static double table_mu(const kpo_dust *d, int j) { return cos(j * PI_ / (d->n_theta - 1)); }

/* 2 pi times the integral of the interpolated S11 over cos Theta (the
 * trapezoid rule, exact for a function linear in cos Theta on each interval) */
static double table_norm(const kpo_dust *d) {
  double sum = 0.0;
  for (int j = 0; j + 1 < d->n_theta; ++j)
    sum += 0.5 * (d->Z[6 * j] + d->Z[6 * (j + 1)]) * (table_mu(d, j) - table_mu(d, j + 1));
  return 2.0 * PI_ * sum;
}

/* the six elements at cos Theta = mu, divided by the normalisation N
 * (bisection for the interval mu_{j+1} <= mu <= mu_j, then linear in mu) */
static void table_at(const kpo_dust *d, double N, double mu, double z[6]) {
  int lo = 0, hi = d->n_theta - 1;
  if (mu > 1.0) mu = 1.0;
  if (mu < -1.0) mu = -1.0;
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (table_mu(d, mid) >= mu) lo = mid; else hi = mid;
  }
  double ma = table_mu(d, lo), mb = table_mu(d, hi);
  double t = ma > mb ? (ma - mu) / (ma - mb) : 0.0;
  for (int k = 0; k < 6; ++k) z[k] = ((1.0 - t) * d->Z[6 * lo + k] + t * d->Z[6 * hi + k]) / N;
}

/* P(m; n) s for tabulated grains: s in the lab basis of n, into the
 * scattering-plane basis (e_par, e_perp) with e_perp = n x m / |n x m| and
 * e_par = e_perp x n (e_perp = phi_hat of n when m = +-n), the block matrix,
 * then from (e_perp x m, e_perp) to the lab basis of m. */
static void table_mueller_lab(const kpo_dust *d, double N, const double m[3], const double n[3],
                              const double s[4], double out[4]) {
  double thn[3], phn[3], thm[3], phm[3], w[3], ep[3], ea[3], eb[3];
  kpo_basis(n, thn, phn);
  kpo_basis(m, thm, phm);
  cross3(n, m, w);
  double w2 = dot3(w, w);
  if (w2 > 1e-24) {
    double r = sqrt(w2);
    for (int k = 0; k < 3; ++k) ep[k] = w[k] / r;
  } else {
    for (int k = 0; k < 3; ++k) ep[k] = phn[k];
  }
  cross3(ep, n, ea);
  double psi = atan2(dot3(ea, phn), dot3(ea, thn));
  double sp[4];
  kpo_rotate_stokes(psi, s, sp);
  double z[6];
  table_at(d, N, dot3(n, m), z);
  double so[4] = {z[0] * sp[0] + z[1] * sp[1], z[1] * sp[0] + z[2] * sp[1],
                  z[3] * sp[2] + z[4] * sp[3], -z[4] * sp[2] + z[5] * sp[3]};
  cross3(ep, m, eb);
  double chi = atan2(dot3(eb, phm), dot3(eb, thm));
  kpo_rotate_stokes(-chi, so, out);
}

/* Cumulative envelope mass over the node intervals (reading T2):
 * cum[0] = 0, cum[j+1] = cum[j] + max(S11_j, S11_{j+1}) / N (mu_j - mu_{j+1}). */
static void table_envelope(const kpo_dust *d, double N, double *cum) {
  cum[0] = 0.0;
  for (int j = 0; j + 1 < d->n_theta; ++j)
    cum[j + 1] = cum[j] + fmax(d->Z[6 * j], d->Z[6 * (j + 1)]) / N * (table_mu(d, j) - table_mu(d, j + 1));
}

static int scatter_event_table(const kpo_dust *d, double N, const double *cum, const double n[3],
                               const double s[4], rng_t *rng, int64_t *trials, double m_out[3],
                               double s_out[4]) {
  double th[3], ph[3];
  kpo_basis(n, th, ph);
  double plin = sqrt(s[1] * s[1] + s[2] * s[2]);
  int nt = d->n_theta;
  for (int trial = 0; trial < 100000; ++trial) {
    double u1 = draw(rng), u2 = draw(rng), u3 = draw(rng), u4 = draw(rng);
    ++*trials;
    double target = u1 * cum[nt - 1];
    int j = 0;
    while (j < nt - 2 && cum[j + 1] <= target) ++j;
    double ma = table_mu(d, j), mb = table_mu(d, j + 1);
    double mu = ma + u2 * (mb - ma);
    double phi = 2.0 * PI_ * u3;
    double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    double m[3];
    for (int k = 0; k < 3; ++k) m[k] = mu * n[k] + st * (cos(phi) * th[k] + sin(phi) * ph[k]);
    double nm = sqrt(dot3(m, m));
    for (int k = 0; k < 3; ++k) m[k] /= nm;
    double o[4];
    table_mueller_lab(d, N, m, n, s, o);
    double env = fmax(d->Z[6 * j], d->Z[6 * (j + 1)]) / N * (s[0] + plin);
    if (o[0] > env * (1.0 + 1e-9)) return -1;
    if (u4 * env <= o[0]) {
      double scale = s[0] / o[0];
      for (int k = 0; k < 4; ++k) s_out[k] = o[k] * scale;
      m_out[0] = m[0]; m_out[1] = m[1]; m_out[2] = m[2];
      return 0;
    }
  }
  return -1;
}

/* ------------------------------------------------------------------------ */
/* Appendix A: analytic solution of the polarised transfer equation across  */
/* one cell with constant coefficients and source (reading R1 for signs).    */
/* The printed I, Q, U, V expressions are evaluated term by term; only the   */
/* exponential factors are formed stably:                                    */
/*   exp(-a1 x) cosh(a2 x) = (exp(-(a1-a2)x) + exp(-(a1+a2)x))/2 (no overflow)*/
/*   1 - that             = -(expm1(-(a1-a2)x) + expm1(-(a1+a2)x))/2         */
/*   exp(-a1 x) sinh(a2 x) = -exp(-(a1-a2)x) expm1(-2 a2 x)/2  (a2 >= 0)       */
/* ------------------------------------------------------------------------ */
void kpo_appA(double a1, double a2, double a3, double dtau,
              const double src[4], const double in[4], double out[4]) {
  double xm = (a1 - a2) * dtau, xp = (a1 + a2) * dtau;
  double x1 = a1 * dtau, x3 = a3 * dtau;
  double em1m = expm1(-xm), em1p = expm1(-xp);
  double Ec = 0.5 * (exp(-xm) + exp(-xp));         /* e^{-a1 x} cosh(a2 x) */
  /* e^{-a1 x} sinh(a2 x), factored so that neither a difference of two tiny
   * exponentials nor an overflowing one is formed */
  double Es = a2 >= 0.0 ? -0.5 * exp(-xm) * expm1(-2.0 * a2 * dtau)
                        : 0.5 * exp(-xp) * expm1(2.0 * a2 * dtau);
  double one_m_Ec = -0.5 * (em1m + em1p);
  double e1 = exp(-x1);
  double Fc = e1 * cos(x3), Fs = e1 * sin(x3);
  double sh = sin(0.5 * x3);
  double one_m_Fc = -expm1(-x1) + e1 * 2.0 * sh * sh;
  double Is = 0.0, Qs = 0.0, Us = 0.0, Vs = 0.0;
  if (src && (src[0] != 0.0 || src[1] != 0.0 || src[2] != 0.0 || src[3] != 0.0)) {
    double D = a1 * a1 - a2 * a2, G = a1 * a1 + a3 * a3;
    Is = (a1 * src[0] - a2 * src[1]) / D;
    Qs = (a1 * src[1] - a2 * src[0]) / D;
    Us = (a1 * src[2] - a3 * src[3]) / G;
    Vs = (a1 * src[3] + a3 * src[2]) / G;
  }
  double I0 = in[0], Q0 = in[1], U0 = in[2], V0 = in[3];
  out[0] = I0 * Ec - Q0 * Es + Is * one_m_Ec + Qs * Es;
  out[1] = -I0 * Es + Q0 * Ec + Qs * one_m_Ec + Is * Es;
  out[2] = U0 * Fc - V0 * Fs + Us * one_m_Fc + Vs * Fs;
  out[3] = U0 * Fs + V0 * Fc + Vs * one_m_Fc - Us * Fs;
}

/* integral_0^len exp(-m s) ds = len * expm1(-m len)/(-m len) */
static double seg_real(double m, double len) {
  double x = -m * len;
  return x == 0.0 ? len : len * expm1(x) / x;
}

/* integral_0^len exp((-m1 + i m3) s) ds */
static double complex seg_cplx(double m1, double m3, double len) {
  double a = -m1 * len, b = m3 * len;
  if (a == 0.0 && b == 0.0) return len;
  double sh = sin(0.5 * b);
  double complex em1 = (expm1(a) * cos(b) - 2.0 * sh * sh) + I * (exp(a) * sin(b));
  return len * em1 / (a + I * b);
}

/* Stokes vector over one straight segment with the scalar split of reading
 * R3: d/ds I = -M I, M = [[m1,m2,0,0],[m2,m1,0,0],[0,0,m1,m3],[0,0,-m3,m1]]
 * (per unit length).  integral = int_0^len exp(-M s) ds in (reading R5),
 * out = exp(-M len) in (Appendix A with zero source). */
void kpo_segment(double m1, double m2, double m3, double len,
                 const double in[4], double integral[4], double out[4]) {
  double gm = seg_real(m1 - m2, len), gp = seg_real(m1 + m2, len);
  double Gc = 0.5 * (gm + gp);   /* int e^{-m1 s} cosh(m2 s) */
  double Gs = 0.5 * (gm - gp);   /* int e^{-m1 s} sinh(m2 s) */
  double complex H = seg_cplx(m1, m3, len);
  double Hc = creal(H), Hs = cimag(H);
  integral[0] = Gc * in[0] - Gs * in[1];
  integral[1] = -Gs * in[0] + Gc * in[1];
  integral[2] = Hc * in[2] - Hs * in[3];
  integral[3] = Hs * in[2] + Hc * in[3];
  kpo_appA(m1, m2, m3, len, NULL, in, out);
}

/* ------------------------------------------------------------------------ */
/* Grid walking: integer cell + offset inside the cell in cell units.        */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t i[3];
  double f[3];
  int64_t leaf;         /* mesh: the leaf block, i[] its local cell; uniform grid: -1 */
} gpos_t;

static int periodic(const kpo_grid *g, int a) { return (g->boundary >> a) & 1; }

/* after crossing a face along `axis`: wrap a periodic axis, or report that
 * the packet left the grid through an open face */
static int leave_or_wrap(const kpo_grid *g, gpos_t *p, int axis) {
  int64_t n = axis == 0 ? g->nx : (axis == 1 ? g->ny : g->nz);
  if (p->i[axis] >= 0 && p->i[axis] < n) return 0;
  if (!periodic(g, axis)) return 1;
  p->i[axis] = p->i[axis] < 0 ? n - 1 : 0;
  return 0;
}

static int inside(const kpo_grid *g, const gpos_t *p) {
  return p->i[0] >= 0 && p->i[0] < g->nx && p->i[1] >= 0 && p->i[1] < g->ny &&
         p->i[2] >= 0 && p->i[2] < g->nz;
}
static int64_t flat(const kpo_grid *g, const gpos_t *p) {
  return p->i[0] + (int64_t)g->nx * (p->i[1] + (int64_t)g->ny * p->i[2]);
}

/* ------------------------------------------------------------------------ */
/* Composite mesh with static refinement (Sec. 2, the mesh the packets       */
/* cross; reading M1).  Positions are kept as (leaf, local cell, fraction);  */
/* on leaving a leaf the point is expressed in units of the finest cell      */
/* (2^-max_level of a root cell) and the leaf holding it is found by         */
/* descending from its root block.                                           */
/* ------------------------------------------------------------------------ */
static double clamp01(double v);

typedef struct {
  int64_t n_leaves;
  int32_t *leaf_of_node;  /* [n_nodes]: leaf id or -1 */
  int64_t *node_of_leaf;  /* [n_leaves] */
  int64_t (*org)[3];      /* [n_leaves]: lower corner in finest cells */
  int32_t *level;         /* [n_leaves] */
  int64_t nfine[3];       /* domain extent in finest cells */
} mesh_ix_t;

static void mesh_free(mesh_ix_t *mx) {
  free(mx->leaf_of_node);
  free(mx->node_of_leaf);
  free(mx->org);
  free(mx->level);
  memset(mx, 0, sizeof *mx);
}

/* Checks the tree (every non-root node the child of exactly one refined
 * node, children after their parent, depth <= max_level) and numbers the
 * leaves in node order with their origins and levels.  0 or -1. */
static int mesh_build(const kpo_grid *g, mesh_ix_t *mx) {
  memset(mx, 0, sizeof *mx);
  const kpo_mesh *m = g->mesh;
  if (!m || !m->child || m->block < 1 || m->max_level < 0 || m->max_level > 20) return -1;
  int64_t R = (int64_t)m->rx * m->ry * m->rz;
  if (m->rx < 1 || m->ry < 1 || m->rz < 1 || m->n_nodes < R) return -1;
  if (g->nx != (int64_t)m->rx * m->block || g->ny != (int64_t)m->ry * m->block ||
      g->nz != (int64_t)m->rz * m->block || g->boundary != 0)
    return -1;
  int32_t N = m->n_nodes;
  int32_t *parents = calloc((size_t)N, sizeof(int32_t));
  int32_t *lev = calloc((size_t)N, sizeof(int32_t));
  int64_t (*org)[3] = calloc((size_t)N, sizeof *org);
  int rc = 0;
  int64_t full = (int64_t)m->block << m->max_level;  /* a root block's edge in finest cells */
  for (int64_t r = 0; r < R; ++r) {
    org[r][0] = (r % m->rx) * full;
    org[r][1] = ((r / m->rx) % m->ry) * full;
    org[r][2] = (r / ((int64_t)m->rx * m->ry)) * full;
  }
  for (int32_t i = 0; i < N && rc == 0; ++i) {
    int32_t c = m->child[i];
    if (c == -1) continue;
    if (c < R || c <= i || (int64_t)c + 8 > N || lev[i] + 1 > m->max_level) { rc = -1; break; }
    int64_t half = full >> (lev[i] + 1);
    for (int k = 0; k < 8; ++k) {
      if (parents[c + k]++) { rc = -1; break; }
      lev[c + k] = lev[i] + 1;
      org[c + k][0] = org[i][0] + ((k & 1) ? half : 0);
      org[c + k][1] = org[i][1] + ((k & 2) ? half : 0);
      org[c + k][2] = org[i][2] + ((k & 4) ? half : 0);
    }
  }
  for (int32_t i = (int32_t)R; i < N && rc == 0; ++i)
    if (parents[i] != 1) rc = -1;
  if (rc == 0) {
    mx->leaf_of_node = malloc(sizeof(int32_t) * (size_t)N);
    for (int32_t i = 0; i < N; ++i) mx->leaf_of_node[i] = m->child[i] == -1 ? (int32_t)mx->n_leaves++ : -1;
    mx->node_of_leaf = malloc(sizeof(int64_t) * (size_t)mx->n_leaves);
    mx->org = malloc(sizeof *mx->org * (size_t)mx->n_leaves);
    mx->level = malloc(sizeof(int32_t) * (size_t)mx->n_leaves);
    for (int32_t i = 0; i < N; ++i) {
      int32_t j = mx->leaf_of_node[i];
      if (j < 0) continue;
      mx->node_of_leaf[j] = i;
      for (int a = 0; a < 3; ++a) mx->org[j][a] = org[i][a];
      mx->level[j] = lev[i];
    }
    mx->nfine[0] = m->rx * full;
    mx->nfine[1] = m->ry * full;
    mx->nfine[2] = m->rz * full;
  }
  free(parents);
  free(lev);
  free(org);
  return rc;
}

/* the leaf holding finest cell X (inside the domain) */
static int64_t mesh_find(const kpo_grid *g, const mesh_ix_t *mx, const int64_t X[3]) {
  const kpo_mesh *m = g->mesh;
  int64_t full = (int64_t)m->block << m->max_level;
  int64_t r[3] = {X[0] / full, X[1] / full, X[2] / full};
  int64_t node = r[0] + m->rx * (r[1] + (int64_t)m->ry * r[2]);
  int64_t o[3] = {r[0] * full, r[1] * full, r[2] * full}, size = full;
  while (m->child[node] != -1) {
    size /= 2;
    int oct = 0;
    for (int a = 0; a < 3; ++a)
      if (X[a] - o[a] >= size) { oct |= 1 << a; o[a] += size; }
    node = m->child[node] + oct;
  }
  return mx->leaf_of_node[node];
}

/* Position t (finest-cell units) in finest cell X -> leaf, local cell, fraction. */
static void mesh_place(const kpo_grid *g, const mesh_ix_t *mx, const double t[3], const int64_t X[3],
                       gpos_t *p) {
  int64_t j = mesh_find(g, mx, X);
  int64_t s = (int64_t)1 << (g->mesh->max_level - mx->level[j]);
  p->leaf = j;
  for (int a = 0; a < 3; ++a) {
    p->i[a] = (X[a] - mx->org[j][a]) / s;
    p->f[a] = clamp01((t[a] - (double)mx->org[j][a]) / (double)s - (double)p->i[a]);
  }
}

/* finest cell of finest-unit coordinate t: a coordinate on a face belongs
 * to the cell the direction points into (R12) */
static int64_t finest_cell(double t, double n) {
  double fl = floor(t);
  int64_t X = (int64_t)fl;
  if (fl == t && n < 0.0) X -= 1;
  return X;
}

/* After cross_face moved the local index of `axis` out of the leaf: the
 * leaf beyond, or 1 if the packet left the domain. */
static int mesh_cross(const kpo_grid *g, const mesh_ix_t *mx, gpos_t *p, const double n[3]) {
  int64_t j = p->leaf;
  double s = (double)((int64_t)1 << (g->mesh->max_level - mx->level[j]));
  double t[3];
  int64_t X[3];
  for (int a = 0; a < 3; ++a) {
    t[a] = (double)mx->org[j][a] + ((double)p->i[a] + p->f[a]) * s;
    X[a] = finest_cell(t[a], n[a]);
    if (X[a] < 0 || X[a] >= mx->nfine[a]) return 1;
  }
  mesh_place(g, mx, t, X, p);
  return 0;
}

/* edge length of the packet's cell */
static double cell_len(const kpo_grid *g, const mesh_ix_t *mx, const gpos_t *p) {
  if (!g->mesh) return g->dx;
  return ldexp(g->dx, -mx->level[p->leaf]);
}

/* flat index of the packet's cell */
static int64_t cell_of(const kpo_grid *g, const gpos_t *p) {
  if (!g->mesh) return flat(g, p);
  int64_t B = g->mesh->block;
  return p->leaf * B * B * B + p->i[0] + B * (p->i[1] + B * p->i[2]);
}

static int64_t cell_count(const kpo_grid *g, const mesh_ix_t *mx) {
  if (!g->mesh) return (int64_t)g->nx * g->ny * g->nz;
  int64_t B = g->mesh->block;
  return mx->n_leaves * B * B * B;
}

/* after cross_face along `axis`: 1 if the packet left the domain */
static int after_cross(const kpo_grid *g, const mesh_ix_t *mx, gpos_t *p, int axis, const double n[3]);

/* Cell holding a point; a coordinate exactly on a face belongs to the cell the
 * direction points into. */
static void locate(const kpo_grid *g, const double x[3], const double n[3], gpos_t *p) {
  double o[3] = {g->x0, g->y0, g->z0};
  for (int a = 0; a < 3; ++a) {
    double t = (x[a] - o[a]) / g->dx;
    double fl = floor(t);
    p->i[a] = (int64_t)fl;
    p->f[a] = t - fl;
    if (p->f[a] == 0.0 && n[a] < 0.0) { p->i[a] -= 1; p->f[a] = 1.0; }
  }
}

/* distance (cell units) to the exit face; ties go to the lowest axis */
static double face_dist(const gpos_t *p, const double n[3], int *axis) {
  double best = INFINITY;
  *axis = -1;
  for (int a = 0; a < 3; ++a) {
    double t;
    if (n[a] > 0.0) t = (1.0 - p->f[a]) / n[a];
    else if (n[a] < 0.0) t = -p->f[a] / n[a];
    else continue;
    if (t < best) { best = t; *axis = a; }
  }
  return best;
}

static double clamp01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

static void move_inside(gpos_t *p, const double n[3], double t) {
  for (int a = 0; a < 3; ++a) p->f[a] = clamp01(p->f[a] + t * n[a]);
}

static void cross_face(gpos_t *p, const double n[3], double t, int axis) {
  for (int a = 0; a < 3; ++a)
    if (a != axis) p->f[a] = clamp01(p->f[a] + t * n[a]);
  if (n[axis] > 0.0) { p->i[axis] += 1; p->f[axis] = 0.0; }
  else { p->i[axis] -= 1; p->f[axis] = 1.0; }
}

static int after_cross(const kpo_grid *g, const mesh_ix_t *mx, gpos_t *p, int axis, const double n[3]) {
  if (!g->mesh) return leave_or_wrap(g, p, axis);
  if (p->i[axis] >= 0 && p->i[axis] < g->mesh->block) return 0;
  return mesh_cross(g, mx, p, n);
}

/* The cell holding point x (direction n for points on faces, R12): 1 if it
 * lies inside the grid, periodic axes wrapped. */
static int locate_in(const kpo_grid *g, const mesh_ix_t *mx, const double x[3], const double n[3],
                     gpos_t *p) {
  p->leaf = -1;
  if (!g->mesh) {
    locate(g, x, n, p);
    for (int a = 0; a < 3; ++a) {
      int64_t na = a == 0 ? g->nx : (a == 1 ? g->ny : g->nz);
      if (periodic(g, a)) p->i[a] = ((p->i[a] % na) + na) % na;
    }
    return inside(g, p);
  }
  double o[3] = {g->x0, g->y0, g->z0}, fine = ldexp(g->dx, -g->mesh->max_level);
  double t[3];
  int64_t X[3];
  for (int a = 0; a < 3; ++a) {
    t[a] = (x[a] - o[a]) / fine;
    X[a] = finest_cell(t[a], n[a]);
    if (X[a] < 0 || X[a] >= mx->nfine[a]) return 0;
  }
  mesh_place(g, mx, t, X, p);
  return 1;
}

static void cell_quat(const float *bhat, int64_t ncell, int64_t c, double q[4]) {
  if (!bhat) { q[0] = 1.0; q[1] = q[2] = q[3] = 0.0; return; }
  double b[3] = {bhat[c], bhat[ncell + c], bhat[2 * ncell + c]};
  kpo_quat_from_b(b, q);
}

static uint64_t fnv_u32(uint64_t h, uint32_t v) {
  for (int k = 0; k < 4; ++k) {
    h ^= (v >> (8 * k)) & 0xffu;
    h *= 1099511628211ULL;
  }
  return h;
}
static uint64_t hash_event(uint64_t h, uint32_t kind, int64_t cell) {
  return fnv_u32(fnv_u32(h, kind), (uint32_t)cell);
}

static void dir_from(double mu, double phi, double n[3]) {
  double s = sqrt(fmax(0.0, 1.0 - mu * mu));
  n[0] = s * cos(phi);
  n[1] = s * sin(phi);
  n[2] = mu;
}

/* Scattering event (Sec. 2.2 and the rejection sampling named in Sec. 3):
 * into the grain frame by quaternion and eta rotation, proposals uniform on
 * the sphere (cos, azimuth, acceptance uniform -- three draws per trial),
 * accept if u * bound <= [P s]_I (reading R6), rescale to the scattered power
 * (reading R7), back to the lab frame.  Returns 0, or -1 if the bound is
 * exceeded or no proposal is accepted within 100000 trials. */
static int scatter_event(const kpo_dust *d, double tab_norm, const double *tab_cum, const double q[4],
                         const double n[3], const double s[4], rng_t *rng, int64_t *trials,
                         double m_out[3], double s_out[4]) {
  if (is_table(d)) return scatter_event_table(d, tab_norm, tab_cum, n, s, rng, trials, m_out, s_out);
  double ng[3], sg[4];
  kpo_to_grain(q, n, ng);
  kpo_rotate_stokes(eta_pair(q, n, ng), s, sg);
  double ap2 = d->a_perp_re * d->a_perp_re + d->a_perp_im * d->a_perp_im;
  double aa2 = d->a_par_re * d->a_par_re + d->a_par_im * d->a_par_im;
  double bound = 3.0 / (8.0 * PI_ * norm_p(d)) * fmax(ap2, aa2) * sg[0];
  double mg[3], og[4];
  int accepted = 0;
  for (int trial = 0; trial < 100000 && !accepted; ++trial) {
    double mu = 2.0 * draw(rng) - 1.0;
    double ph = 2.0 * PI_ * draw(rng);
    double ua = draw(rng);
    ++*trials;
    dir_from(mu, ph, mg);
    mueller_grain(d, mg, ng, sg, og);
    if (og[0] > bound * (1.0 + 1e-12)) return -1;
    if (ua * bound <= og[0]) accepted = 1;
  }
  if (!accepted) return -1;
  double scale = scatter_weight_grain(d, ng, sg) / og[0];
  for (int k = 0; k < 4; ++k) og[k] *= scale;
  double m[3];
  kpo_from_grain(q, mg, m);
  kpo_rotate_stokes(-eta_pair(q, m, mg), og, s_out);
  m_out[0] = m[0]; m_out[1] = m[1]; m_out[2] = m[2];
  return 0;
}

int kpo_scatter_sample(const kpo_dust *d, const double q[4], const double n[3],
                       const double s[4], uint64_t seed, uint64_t lam, uint64_t packet,
                       uint64_t first_draw, double m_out[3], double s_out[4],
                       int64_t *trials) {
  rng_t r = {{seed, lam}, packet, first_draw, 0, 0, {0, 0, 0, 0}};
  *trials = 0;
  double *cum = NULL, N = 0.0;
  if (is_table(d)) {
    N = table_norm(d);
    cum = malloc(sizeof(double) * (size_t)d->n_theta);
    table_envelope(d, N, cum);
  }
  int rc = scatter_event(d, N, cum, q, n, s, &r, trials, m_out, s_out);
  free(cum);
  return rc;
}

typedef struct {
  const kpo_grid *g;
  const float *rho, *bhat;
  const kpo_dust *d;
  const kpo_source *src;
  const kpo_opts *o;
  int32_t lam;
  uint64_t n_total;
  int32_t n_views;
  const kpo_view *views;
  double (*vdir)[3];     /* camera directions */
  double *S;             /* [cell][view][4] or NULL */
  const double *cdf;     /* thermal emission: running sum of cell luminosities */
  double *peel;          /* peel-off images [view][4][npy][npx] or NULL */
  double tab_norm;       /* tabulated scattering: 2 pi times the integral of S11 over cos Theta */
  const double *tab_cum; /* ... and the cumulative envelope mass [n_theta] */
  const mesh_ix_t *mx;   /* the mesh's leaf table (unused on a uniform grid) */
  int64_t ncell;
} run_t;

/* P(m; n) s (lab bases) with the run's table normalisation */
static void mueller_run(const run_t *R, const double q[4], const double m[3], const double n[3],
                        const double s[4], double out[4]) {
  if (is_table(R->d)) table_mueller_lab(R->d, R->tab_norm, m, n, s, out);
  else kpo_mueller_lab(R->d, q, m, n, s, out);
}

/* Running sum over cells (flat order) of the thermal luminosity
 * 4 pi rho kappa_abs B V of each cell (reading E1); NULL if it is zero. */
static double *emission_cdf(const kpo_grid *g, const mesh_ix_t *mx, const float *rho, const kpo_dust *d,
                            const float *B) {
  int64_t ncell = cell_count(g, mx);
  double *cdf = malloc(sizeof(double) * (size_t)ncell);
  if (!cdf) return NULL;
  double run = 0.0;
  int64_t B3 = g->mesh ? (int64_t)g->mesh->block * g->mesh->block * g->mesh->block : 1;
  for (int64_t c = 0; c < ncell; ++c) {
    double len = g->mesh ? ldexp(g->dx, -mx->level[c / B3]) : g->dx;  /* the cell's edge (M1) */
    double vol = len * len * len;
    run += 4.0 * PI_ * (double)rho[c] * d->kappa_abs * (double)B[c] * vol;
    cdf[c] = run;
  }
  if (!(run > 0.0) || !isfinite(run)) { free(cdf); return NULL; }
  return cdf;
}

double kpo_emission_luminosity(const kpo_grid *g, const float *rho, const kpo_dust *d,
                               const float *B) {
  mesh_ix_t mx;
  memset(&mx, 0, sizeof mx);
  if (g->mesh && mesh_build(g, &mx)) { mesh_free(&mx); return 0.0; }
  double *cdf = emission_cdf(g, &mx, rho, d, B);
  double L = cdf ? cdf[cell_count(g, &mx) - 1] : 0.0;
  free(cdf);
  mesh_free(&mx);
  return L;
}

/* The emitting cell of a uniform u: the first cell whose running sum
 * exceeds u L (so a cell of zero luminosity is never drawn). */
static int64_t emission_cell(const double *cdf, int64_t ncell, double u) {
  double t = u * cdf[ncell - 1];
  int64_t lo = 0, hi = ncell - 1;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (t < cdf[mid]) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

/* Thermal emission of one packet of weight w (Sec. 2.2, reading E1): the
 * cell drawn by luminosity, the position uniform inside it, the direction
 * isotropic, the Stokes vector w (alpha1, alpha2, 0, 0) in the grain-frame
 * basis of the direction carried to the lab basis (mean over directions w,
 * the orientation average of alpha1 being 1).  Draws: cell, three
 * coordinates, two for the direction. */
static void emit_thermal(const kpo_grid *g, const mesh_ix_t *mx, const float *bhat, const kpo_dust *d,
                         const double *cdf, rng_t *rng, double w, gpos_t *p, double n[3],
                         double s[4]) {
  int64_t ncell = cell_count(g, mx);
  int64_t c = emission_cell(cdf, ncell, draw(rng));
  if (g->mesh) {
    /* cell c of the mesh: leaf c / block^3, local cell x fastest (M1) */
    int64_t Bk = g->mesh->block, r = c % (Bk * Bk * Bk);
    p->leaf = c / (Bk * Bk * Bk);
    p->i[0] = r % Bk;
    p->i[1] = (r / Bk) % Bk;
    p->i[2] = r / (Bk * Bk);
  } else {
    p->leaf = -1;
    p->i[0] = c % g->nx;
    p->i[1] = (c / g->nx) % g->ny;
    p->i[2] = c / ((int64_t)g->nx * g->ny);
  }
  for (int a = 0; a < 3; ++a) p->f[a] = draw(rng);
  double mu = 2.0 * draw(rng) - 1.0;
  double ph = 2.0 * PI_ * draw(rng);
  dir_from(mu, ph, n);
  double q[4], ng[3], al[3];
  cell_quat(bhat, ncell, c, q);
  kpo_to_grain(q, n, ng);
  kpo_alphas(d, ng[2], al);
  double sg[4] = {w * al[0], w * al[1], 0.0, 0.0};
  kpo_rotate_stokes(-eta_pair(q, n, ng), sg, s);
}

int kpo_emit_state(const kpo_grid *g, const float *rho, const float *bhat,
                   const kpo_dust *d, const float *B, uint64_t seed, int32_t lam,
                   uint64_t packet, double w, int64_t *cell, double pos[3], double n[3],
                   double s[4]) {
  if (!g || !rho || !d || !B) return -1;
  mesh_ix_t mx;
  memset(&mx, 0, sizeof mx);
  if (g->mesh && mesh_build(g, &mx)) { mesh_free(&mx); return -1; }
  double *cdf = emission_cdf(g, &mx, rho, d, B);
  if (!cdf) { mesh_free(&mx); return -1; }
  rng_t rng = {{seed, (uint64_t)lam}, packet, 0, 0, 0, {0, 0, 0, 0}};
  gpos_t p;
  emit_thermal(g, &mx, bhat, d, cdf, &rng, w, &p, n, s);
  free(cdf);
  mesh_free(&mx);
  *cell = cell_of(g, &p);
  for (int a = 0; a < 3; ++a) pos[a] = p.f[a];
  return 0;
}

static void atomic_add(double *p, double v) {
#pragma omp atomic
  *p += v;
}

/* Peel-off imaging at a scattering event (the Monte Carlo imaging Sec. 2.3
 * compares two-step imaging with): for every camera, the Stokes vector the
 * event scatters toward it per unit solid angle, P(Omega_v; n) s in the
 * camera basis (the normalised Mueller matrix of reading R5), carried to the
 * grid's edge through the Appendix A extinction of every cell on the way
 * (no source), and added to the pixel the event projects to, divided by the
 * pixel's area (reading R9 for the camera).  Open boundaries. */
static void peel_off(const run_t *R, const gpos_t *at, const double q_ev[4], const double n[3],
                     const double s[4]) {
  const kpo_grid *g = R->g;
  const kpo_dust *d = R->d;
  int64_t ncell = R->ncell;
  double kext = d->kappa_sca + d->kappa_abs;
  double X[3] = {g->x0 + (at->i[0] + at->f[0]) * g->dx, g->y0 + (at->i[1] + at->f[1]) * g->dx,
                 g->z0 + (at->i[2] + at->f[2]) * g->dx};
  if (g->mesh) {
    /* the event's position: its leaf's corner plus the local cell and
     * fraction, in finest cells (M1) */
    const mesh_ix_t *mx = R->mx;
    double s = (double)((int64_t)1 << (g->mesh->max_level - mx->level[at->leaf]));
    double fine = ldexp(g->dx, -g->mesh->max_level), o[3] = {g->x0, g->y0, g->z0};
    for (int a = 0; a < 3; ++a)
      X[a] = o[a] + ((double)mx->org[at->leaf][a] + ((double)at->i[a] + at->f[a]) * s) * fine;
  }
  int32_t npx = R->views[0].npx, npy = R->views[0].npy;
  for (int v = 0; v < R->n_views; ++v) {
    const double *om = R->vdir[v];
    double th[3], ph[3];
    kpo_basis(om, th, ph);
    double W = R->views[v].half_width;
    double xi = dot3(X, ph), yi = -dot3(X, th);
    double fx = (xi + W) / (2.0 * W / npx), fy = (yi + W) / (2.0 * W / npy);
    if (!(fx >= 0.0 && fx < npx && fy >= 0.0 && fy < npy)) continue;
    int ix = (int)fx, iy = (int)fy;
    double st[4];
    mueller_run(R, q_ev, om, n, s, st);
    gpos_t p = *at;
    while (1) {
      int axis;
      double tf = face_dist(&p, om, &axis);
      if (axis < 0) break;
      int64_t c = cell_of(g, &p);
      double r = (double)R->rho[c];
      if (r > 0.0 && tf > 0.0) {
        double q[4], og[3], al[3], sg[4], out[4], zero[4] = {0, 0, 0, 0};
        cell_quat(R->bhat, ncell, c, q);
        kpo_to_grain(q, om, og);
        kpo_alphas(d, og[2], al);
        double eta = eta_pair(q, om, og);
        kpo_rotate_stokes(eta, st, sg);
        kpo_appA(al[0], al[1], al[2], r * kext * tf * cell_len(g, R->mx, &p), zero, sg, out);
        kpo_rotate_stokes(-eta, out, st);
      }
      cross_face(&p, om, tf, axis);
      if (after_cross(g, R->mx, &p, axis, om)) break;
    }
    double area = (2.0 * W / npx) * (2.0 * W / npy);
    for (int k = 0; k < 4; ++k)
      atomic_add(R->peel + (((int64_t)v * 4 + k) * npy + iy) * npx + ix, st[k] / area);
  }
}

/* One packet from emission to termination (Sec. 2.2-2.3). */
static void run_packet(const run_t *R, uint64_t pid, kpo_trace *tr, kpo_stats *st) {
  const kpo_grid *g = R->g;
  const kpo_dust *d = R->d;
  int64_t ncell = R->ncell;
  double kext = d->kappa_sca + d->kappa_abs;
  rng_t rng = {{R->o->seed, (uint64_t)R->lam}, pid, 0, 0, 0, {0, 0, 0, 0}};

  /* emission: a point source (isotropic unpolarised or pencil) or the dust's
   * thermal emission (reading E1), then an exponential scattering depth */
  double n[3], s[4], w0;
  gpos_t p;
  int in = 1;
  if (R->src->kind == 2) {
    w0 = R->cdf[ncell - 1] / (double)R->n_total;
    emit_thermal(g, R->mx, R->bhat, d, R->cdf, &rng, w0, &p, n, s);
  } else {
    double u0 = draw(&rng), u1 = draw(&rng);
    if (R->src->kind == 1) {
      double nn = sqrt(dot3(R->src->dir, R->src->dir));
      for (int a = 0; a < 3; ++a) n[a] = R->src->dir[a] / nn;
    } else {
      dir_from(2.0 * u0 - 1.0, 2.0 * PI_ * u1, n);
    }
    w0 = R->src->lum / (double)R->n_total;
    s[0] = w0; s[1] = s[2] = s[3] = 0.0;
    in = locate_in(g, R->mx, R->src->pos, n, &p);
  }
  double tau = -log(draw(&rng));
  st->e_emitted += s[0];

  int32_t events = 0, end = KPO_END_NONE;
  int64_t steps = 0, last = -1;
  double tau_path = 0.0;
  uint64_t h = 14695981039346656037ULL;
  if (!in) {
    end = KPO_END_ESCAPE;
    st->escaped++;
    st->e_escaped += s[0];
  }
  while (end == KPO_END_NONE) {
    int64_t c = cell_of(g, &p);
    double clen = cell_len(g, R->mx, &p), vol = clen * clen * clen;
    last = c;
    if (events >= R->o->max_events || steps >= KPO_MAX_STEPS) {
      h = hash_event(h, KPO_END_BUDGET, c);
      end = KPO_END_BUDGET;
      st->budget++;
      st->e_budget += s[0];
      break;
    }
    int axis;
    double tf = face_dist(&p, n, &axis);
    if (axis < 0 || !isfinite(tf)) { end = KPO_END_NUMERIC; st->numeric++; break; }
    double rho = (double)R->rho[c];
    double kbar = rho * d->kappa_sca, ke = rho * kext;
    double lface = tf * clen, len;
    int scat;
    if (kbar > 0.0 && tau < kbar * lface) { len = tau / kbar; scat = 1; }
    else { len = lface; tau -= kbar * lface; scat = 0; }
    steps++;
    st->cell_steps++;

    double q[4];
    cell_quat(R->bhat, ncell, c, q);
    if (rho > 0.0 && len > 0.0) {
      /* extinction across the segment in the grain frame (Sec. 2.2, App. A) */
      double ng[3], al[3], sg[4], jg[4], og[4], jl[4];
      kpo_to_grain(q, n, ng);
      kpo_alphas(d, ng[2], al);
      double eta = eta_pair(q, n, ng);
      kpo_rotate_stokes(eta, s, sg);
      kpo_segment(ke * al[0] - kbar, ke * al[1], ke * al[2], len, sg, jg, og);
      tau_path += fabs(ke * al[0] - kbar) * len;
      kpo_rotate_stokes(-eta, jg, jl);
      double I_before = s[0];
      kpo_rotate_stokes(-eta, og, s);
      st->e_absorbed += I_before - s[0];
      /* scattering source tally, every segment (Sec. 2.3, reading R5) */
      if (R->S && kbar > 0.0) {
        for (int v = 0; v < R->n_views; ++v) {
          double pv[4];
          mueller_run(R, q, R->vdir[v], n, jl, pv);
          double *dst = R->S + (c * R->n_views + v) * 4;
          for (int k = 0; k < 4; ++k) atomic_add(dst + k, kbar / vol * pv[k]);
        }
      }
    }

    if (scat) {
      move_inside(&p, n, len / clen);
      if (R->peel) peel_off(R, &p, q, n, s);
      double m[3], i_in = s[0];
      if (scatter_event(d, R->tab_norm, R->tab_cum, q, n, s, &rng, &st->trials, m, s) != 0) {
        end = KPO_END_NUMERIC;
        st->numeric++;
        break;
      }
      n[0] = m[0]; n[1] = m[1]; n[2] = m[2];
      st->e_scat_delta += s[0] - i_in;
      events++;
      st->scatterings++;
      h = hash_event(h, KPO_EV_SCATTER, c);
      tau = -log(draw(&rng));
    } else {
      cross_face(&p, n, tf, axis);
      if (after_cross(g, R->mx, &p, axis, n)) {
        h = hash_event(h, KPO_END_ESCAPE, c);
        end = KPO_END_ESCAPE;
        st->escaped++;
        st->e_escaped += s[0];
        break;
      }
    }
    if (!isfinite(s[0])) { end = KPO_END_NUMERIC; st->numeric++; break; }
    /* Russian roulette (reading R8) */
    if (R->o->rr_wmin > 0.0 && s[0] < R->o->rr_wmin * w0) {
      double u = draw(&rng);
      if (u < R->o->rr_psurv) {
        double before = s[0];
        for (int k = 0; k < 4; ++k) s[k] /= R->o->rr_psurv;
        st->rr_survivals++;
        st->e_rr_gained += s[0] - before;
        h = hash_event(h, KPO_EV_RR_SURVIVE, cell_of(g, &p));
      } else {
        st->rr_kills++;
        st->e_rr_killed += s[0];
        h = hash_event(h, KPO_END_RR_KILL, cell_of(g, &p));
        end = KPO_END_RR_KILL;
        break;
      }
    }
  }
  if (tr) {
    tr->packet = pid;
    tr->end_kind = end;
    tr->events = events;
    tr->steps = steps;
    tr->last_cell = last;
    for (int a = 0; a < 3; ++a) tr->n[a] = n[a];
    for (int k = 0; k < 4; ++k) tr->stokes[k] = s[k];
    tr->hash = h;
    tr->tau_path = tau_path;
  }
}

static void view_dir(const kpo_view *v, double out[3]) {
  out[0] = sin(v->theta) * cos(v->phi);
  out[1] = sin(v->theta) * sin(v->phi);
  out[2] = cos(v->theta);
}

static void stats_add(kpo_stats *a, const kpo_stats *b) {
  a->cell_steps += b->cell_steps; a->scatterings += b->scatterings; a->trials += b->trials;
  a->rr_kills += b->rr_kills; a->rr_survivals += b->rr_survivals; a->escaped += b->escaped;
  a->budget += b->budget; a->numeric += b->numeric;
  a->e_emitted += b->e_emitted; a->e_escaped += b->e_escaped; a->e_absorbed += b->e_absorbed;
  a->e_rr_killed += b->e_rr_killed; a->e_rr_gained += b->e_rr_gained; a->e_budget += b->e_budget;
  a->e_scat_delta += b->e_scat_delta;
}

static int check_inputs(const kpo_grid *g, const kpo_dust *d, const kpo_source *src) {
  if (!g || !d || !src) return -1;
  if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0 || !(g->dx > 0.0)) return -1;
  if (!(d->kappa_sca >= 0.0) || !(d->kappa_abs >= 0.0)) return -1;
  if (!is_sphere(d) && !(2.0 * d->a_perp_im + d->a_par_im > 0.0)) return -1;
  if (d->n_theta != 0) {
    if (d->n_theta < 2 || !d->Z) return -1;
    for (int j = 0; j < d->n_theta; ++j)
      for (int k = 0; k < 6; ++k)
        if (!isfinite(d->Z[6 * j + k]) || fabs(d->Z[6 * j + k]) > d->Z[6 * j]) return -1;
    if (!(table_norm(d) > 0.0)) return -1;
  }
  if (src->kind != 0 && src->kind != 1 && src->kind != 2) return -1;
  if (src->kind == 2 && !src->B) return -1;
  return 0;
}

static int transport_impl(const kpo_grid *g, const float *rho, const float *bhat,
                          const kpo_dust *d, int32_t lam, const kpo_source *src,
                          int32_t n_views, const kpo_view *views,
                          uint64_t p_begin, uint64_t p_end, uint64_t n_total,
                          const kpo_opts *o, double *S, kpo_trace *traces, double *peel,
                          kpo_stats *stats) {
  if (check_inputs(g, d, src) || !o || n_total == 0 || p_end < p_begin) return -1;
  if ((S || peel) && (n_views <= 0 || !views)) return -1;
  if (peel && g->boundary != 0) return -1;
  mesh_ix_t mx;
  memset(&mx, 0, sizeof mx);
  if (g->mesh && mesh_build(g, &mx)) { mesh_free(&mx); return -1; }
  double *cdf = NULL;
  if (src->kind == 2 && !(cdf = emission_cdf(g, &mx, rho, d, src->B))) { mesh_free(&mx); return -1; }
  double (*vdir)[3] = NULL;
  if (n_views > 0) {
    vdir = malloc(sizeof(double[3]) * (size_t)n_views);
    for (int v = 0; v < n_views; ++v) view_dir(&views[v], vdir[v]);
  }
  double *cum = NULL, N = 0.0;
  if (is_table(d)) {
    N = table_norm(d);
    cum = malloc(sizeof(double) * (size_t)d->n_theta);
    table_envelope(d, N, cum);
  }
  run_t R = {g, rho, bhat, d, src, o, lam, n_total, n_views, views, vdir, S, cdf, peel, N, cum,
             &mx, cell_count(g, &mx)};
  kpo_stats total;
  memset(&total, 0, sizeof total);
  int nth = o->nthreads;
#pragma omp parallel num_threads(nth > 0 ? nth : omp_get_max_threads())
  {
    kpo_stats local;
    memset(&local, 0, sizeof local);
#pragma omp for schedule(dynamic, 16)
    for (int64_t k = 0; k < (int64_t)(p_end - p_begin); ++k)
      run_packet(&R, p_begin + (uint64_t)k, traces ? &traces[k] : NULL, &local);
#pragma omp critical
    stats_add(&total, &local);
  }
  if (stats) stats_add(stats, &total);
  free(vdir);
  free(cdf);
  free(cum);
  mesh_free(&mx);
  return 0;
}

int kpo_transport(const kpo_grid *g, const float *rho, const float *bhat,
                  const kpo_dust *d, int32_t lam, const kpo_source *src,
                  int32_t n_views, const kpo_view *views,
                  uint64_t p_begin, uint64_t p_end, uint64_t n_total,
                  const kpo_opts *o, double *S, kpo_trace *traces,
                  kpo_stats *stats) {
  return transport_impl(g, rho, bhat, d, lam, src, n_views, views, p_begin, p_end, n_total, o, S,
                        traces, NULL, stats);
}

int kpo_transport_peel(const kpo_grid *g, const float *rho, const float *bhat,
                       const kpo_dust *d, int32_t lam, const kpo_source *src,
                       int32_t n_views, const kpo_view *views,
                       uint64_t p_begin, uint64_t p_end, uint64_t n_total,
                       const kpo_opts *o, double *S, double *peel, kpo_stats *stats) {
  if (!peel) return -1;
  return transport_impl(g, rho, bhat, d, lam, src, n_views, views, p_begin, p_end, n_total, o, S,
                        NULL, peel, stats);
}

int kpo_trace_packets(const kpo_grid *g, const float *rho, const float *bhat,
                      const kpo_dust *d, int32_t lam, const kpo_source *src,
                      const uint64_t *ids, uint64_t n_ids, uint64_t n_total,
                      const kpo_opts *o, kpo_trace *traces) {
  if (check_inputs(g, d, src) || !o || !ids || !traces || n_total == 0) return -1;
  mesh_ix_t mx;
  memset(&mx, 0, sizeof mx);
  if (g->mesh && mesh_build(g, &mx)) { mesh_free(&mx); return -1; }
  double *cdf = NULL;
  if (src->kind == 2 && !(cdf = emission_cdf(g, &mx, rho, d, src->B))) { mesh_free(&mx); return -1; }
  double *cum = NULL, N = 0.0;
  if (is_table(d)) {
    N = table_norm(d);
    cum = malloc(sizeof(double) * (size_t)d->n_theta);
    table_envelope(d, N, cum);
  }
  run_t R = {g, rho, bhat, d, src, o, lam, n_total, 0, NULL, NULL, NULL, cdf, NULL, N, cum,
             &mx, cell_count(g, &mx)};
  int nth = o->nthreads;
#pragma omp parallel num_threads(nth > 0 ? nth : omp_get_max_threads())
  {
    kpo_stats local;
    memset(&local, 0, sizeof local);
#pragma omp for schedule(dynamic, 4)
    for (int64_t k = 0; k < (int64_t)n_ids; ++k) run_packet(&R, ids[k], &traces[k], &local);
  }
  free(cdf);
  free(cum);
  mesh_free(&mx);
  return 0;
}

int kpo_image(const kpo_grid *g, const float *rho, const float *bhat,
              const kpo_dust *d, int32_t n_views, const kpo_view *views,
              const double *S, double *images) {
  if (!S) return -1;
  return kpo_image_thermal(g, rho, bhat, d, n_views, views, S, NULL, images);
}

/* Step 2 of two-step imaging (Sec. 2.3): march each pixel ray across the
 * grid toward the camera, solving Appendix A cell by cell with the source
 * S/(rho kappa_ext) per unit optical depth (reading R9 for the camera), plus
 * the dust's thermal emission (kappa_abs/kappa_ext)(alpha1, alpha2, 0, 0) B
 * per unit optical depth in the grain-frame basis (eq. polarized-rt, E1). */
int kpo_image_thermal(const kpo_grid *g, const float *rho, const float *bhat,
                      const kpo_dust *d, int32_t n_views, const kpo_view *views,
                      const double *S, const float *B, double *images) {
  kpo_source dummy = {0, {0, 0, 0}, {0, 0, 1}, 1.0, NULL};
  if (check_inputs(g, d, &dummy) || n_views <= 0 || !views || !images) return -1;
  mesh_ix_t mx;
  memset(&mx, 0, sizeof mx);
  if (g->mesh && mesh_build(g, &mx)) { mesh_free(&mx); return -1; }
  int64_t ncell = cell_count(g, &mx);
  double fine = g->mesh ? ldexp(g->dx, -g->mesh->max_level) : g->dx;
  double kext = d->kappa_sca + d->kappa_abs;
  double lo[3] = {g->x0, g->y0, g->z0};
  double hi[3] = {g->x0 + g->nx * g->dx, g->y0 + g->ny * g->dx, g->z0 + g->nz * g->dx};
  int32_t npx = views[0].npx, npy = views[0].npy;
  for (int v = 0; v < n_views; ++v)
    if (views[v].npx != npx || views[v].npy != npy || npx <= 0 || npy <= 0) return -1;
  for (int v = 0; v < n_views; ++v) {
    double om[3];
    view_dir(&views[v], om);
    /* a ray must leave through an open face within KPO_MAX_STEPS cell
     * lengths (reading R14): its path through the open extent is at most
     * n_a / |om_a| cells for every open axis a */
    int64_t nn[3] = {g->nx, g->ny, g->nz};
    double cells = INFINITY;
    for (int a = 0; a < 3; ++a)
      if (!periodic(g, a) && om[a] != 0.0) cells = fmin(cells, (double)nn[a] / fabs(om[a]));
    if (!(cells <= (double)KPO_MAX_STEPS)) { mesh_free(&mx); return -1; }
  }
  for (int v = 0; v < n_views; ++v) {
    double om[3], th[3], ph[3];
    view_dir(&views[v], om);
    kpo_basis(om, th, ph);
    double W = views[v].half_width;
#pragma omp parallel for schedule(dynamic, 8) collapse(2)
    for (int iy = 0; iy < npy; ++iy)
      for (int ix = 0; ix < npx; ++ix) {
        double xp = -W + (ix + 0.5) * (2.0 * W / npx);
        double yp = -W + (iy + 0.5) * (2.0 * W / npy);
        double P0[3];
        for (int a = 0; a < 3; ++a) P0[a] = xp * ph[a] - yp * th[a];
        double sn = -INFINITY, sf = INFINITY;
        int miss = 0;
        for (int a = 0; a < 3; ++a) {
          if (periodic(g, a)) continue;  /* the copies fill the axis */
          if (om[a] != 0.0) {
            double s1 = (lo[a] - P0[a]) / om[a], s2 = (hi[a] - P0[a]) / om[a];
            sn = fmax(sn, fmin(s1, s2));
            sf = fmin(sf, fmax(s1, s2));
          } else if (P0[a] < lo[a] || P0[a] >= hi[a]) {
            miss = 1;
          }
        }
        double st[4] = {0, 0, 0, 0};
        if (!miss && sn < sf) {
          gpos_t p;
          p.leaf = -1;
          int64_t nn[3] = {g->nx, g->ny, g->nz};
          if (g->mesh) {
            /* the entry point in finest cells, clamped into the domain */
            double t[3];
            int64_t X[3];
            for (int a = 0; a < 3; ++a) {
              t[a] = (P0[a] + sn * om[a] - lo[a]) / fine;
              X[a] = (int64_t)floor(t[a]);
              if (X[a] < 0) X[a] = 0;
              if (X[a] > mx.nfine[a] - 1) X[a] = mx.nfine[a] - 1;
            }
            mesh_place(g, &mx, t, X, &p);
          }
          for (int a = 0; a < 3 && !g->mesh; ++a) {
            double t = (P0[a] + sn * om[a] - lo[a]) / g->dx;
            double fl = floor(t);
            int64_t i = (int64_t)fl;
            if (periodic(g, a)) {
              p.i[a] = ((i % nn[a]) + nn[a]) % nn[a];
              p.f[a] = clamp01(t - fl);
              continue;
            }
            if (i < 0) i = 0;
            if (i > nn[a] - 1) i = nn[a] - 1;
            p.i[a] = i;
            p.f[a] = clamp01(t - (double)i);
          }
          while (1) {
            int axis;
            double tf = face_dist(&p, om, &axis);
            if (axis < 0) break;
            int64_t c = cell_of(g, &p);
            double clen = cell_len(g, &mx, &p);
            double r = (double)rho[c];
            if (r > 0.0) {
              double ke = r * kext, q[4], og[3], al[3], sg[4], srcg[4], src[4];
              cell_quat(bhat, ncell, c, q);
              kpo_to_grain(q, om, og);
              kpo_alphas(d, og[2], al);
              double eta = eta_pair(q, om, og);
              for (int k = 0; k < 4; ++k) src[k] = S ? S[(c * n_views + v) * 4 + k] / ke : 0.0;
              kpo_rotate_stokes(eta, st, sg);
              kpo_rotate_stokes(eta, src, srcg);
              if (B) {
                double e = d->kappa_abs / kext * (double)B[c];
                srcg[0] += e * al[0];
                srcg[1] += e * al[1];
              }
              double out[4];
              kpo_appA(al[0], al[1], al[2], ke * tf * clen, srcg, sg, out);
              kpo_rotate_stokes(-eta, out, st);
            }
            cross_face(&p, om, tf, axis);
            if (after_cross(g, &mx, &p, axis, om)) break;
          }
        }
        for (int k = 0; k < 4; ++k)
          images[(((int64_t)v * 4 + k) * npy + iy) * npx + ix] = st[k];
      }
  }
  mesh_free(&mx);
  return 0;
}
