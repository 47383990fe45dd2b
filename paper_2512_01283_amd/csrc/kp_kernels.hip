// kp_kernels.hip -- gfx950 kernels of the polarized Monte Carlo transport
// (step 1) and the deterministic imaging ray-march (step 2) of Yang & Wang,
// arXiv:2512.01283, Sec. 2.2-2.3 and Appendix A.
//
// Step 1 is a persistent packet-per-lane loop: every lane of a 64-wide
// wavefront carries one photon packet and advances it by one cell segment per
// iteration (plus the scattering event that may end the segment); lanes whose
// packet ended are refilled from a global work counter once per iteration
// (one atomic per wavefront, ids handed out by lane rank), so long and short
// paths do not idle a wavefront.  Packets are independent: each draws from its
// own Philox stream (key (seed, wavelength), counter (packet, block, 0, 0)),
// so the schedule never changes a packet's path.
//
// The scattering-source tally of step 1 is kept as the incident coherency of
// each cell (3x3 Hermitian, 9 reals): because every scatterer here is a
// dipole, the source toward any camera is a fixed linear map of it (formed in
// step 2), so one tally serves all views and wavelengths' views at 9 FP64
// atomics per segment instead of 4 per view (6 when no circular polarisation
// can arise, i.e. for spheres).  A lane keeps the running sum for its current
// cell in registers and hands it over only when it moves to another cell
// (multiple scattering inside a thick cell costs no atomics).  Hand-overs are
// flushed cooperatively by the whole wavefront: the pending sums are staged in
// LDS and re-issued so that one atomic instruction carries the contiguous
// components of ~7-10 cells, each cell's block aligned to one cache line
// (64 B for 6 reals, 128 B for 9) -- memory-side FP64 atomics are charged per
// line request, so this is ~5x cheaper than one cell per lane.
#include "kp_device.hpp"
#include "kp_internal.hpp"

namespace kp {

enum : uint32_t {
  EV_SCATTER = 1, END_ESCAPE = 2, EV_RR_SURVIVE = 3, END_RR_KILL = 4, END_BUDGET = 5,
  END_NUMERIC = 6
};

__device__ __forceinline__ uint64_t fnv_u32(uint64_t h, uint32_t v) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    h ^= (v >> (8 * k)) & 0xffu;
    h *= 1099511628211ull;
  }
  return h;
}
__device__ __forceinline__ uint64_t hash_event(uint64_t h, uint32_t kind, uint64_t cell) {
  return fnv_u32(fnv_u32(h, kind), (uint32_t)cell);
}

template <typename R> struct Cx { R re, im; };
template <typename R> __device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R> __device__ __forceinline__ Cx<R> cmulc(Cx<R> a, Cx<R> b) {  // a * conj(b)
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename R> __device__ __forceinline__ Cx<R> cadd(Cx<R> a, Cx<R> b) {
  return {a.re + b.re, a.im + b.im};
}
template <typename R> __device__ __forceinline__ R cabs2(Cx<R> a) { return a.re * a.re + a.im * a.im; }
template <typename R> __device__ __forceinline__ Cx<R> cscale(Cx<R> a, R s) { return {a.re * s, a.im * s}; }

template <typename R>
struct Packet {
  // Geometry is FP64 in every variant: position inside the cell (cell units),
  // direction and remaining scattering depth.  A packet's path is sensitive
  // to them well beyond their own size -- a scattering depth off by 3e-7
  // moves a scattering point inside a tenuous cell (rho kappa dx ~ 1e-3) by
  // 3e-4 cell, which a later cell of optical depth 1e3 turns into a 0.3 %
  // weight error -- so only the polarisation arithmetic runs in R.
  double fx, fy, fz;
  double nx, ny, nz;
  double rnx, rny, rnz;  // 1 / n per axis (inf for a zero component), set with n
  double tau;
  R I, Q, U, V;       // Stokes vector in the lab basis of n
  R w0;               // initial weight
  R tau_path;         // sum of |continuous extinction exponent| along the path
  R u0, u1, u2, u3;   // uniforms of the Philox block `blk`
  double e_abs, e_scat, e_gain;
  double ks, ke;      // per-wavelength kappa_sca and kappa_ext times the cell size, held
  R ka;               // in registers (no dependent load per step); ka = kappa_abs dx
  float rho;          // density of the current cell when the grid holds it (loaded on
                      // entering the cell, one step before its use)
  uint64_t pid, hash;
  int64_t last;
  int ci, cj, ck;
  int leaf, lvl;      // composite mesh: the leaf block (ci..ck local to it) and its level
  uint32_t draw, blk;
  int events, steps, trials, lam, rr;
};

template <typename R>
__device__ __forceinline__ R next_uniform(Packet<R>& p, uint64_t seed) {
  uint32_t d = p.draw++;
  uint32_t b = d >> 2;
  if (b != p.blk) {
    uint64_t w[4];
    philox4x64_10(p.pid, (uint64_t)b, 0ull, 0ull, seed, (uint64_t)p.lam, w);
    p.u0 = word_uniform<R>(w[0]);
    p.u1 = word_uniform<R>(w[1]);
    p.u2 = word_uniform<R>(w[2]);
    p.u3 = word_uniform<R>(w[3]);
    p.blk = b;
  }
  uint32_t k = d & 3u;
  return k == 0 ? p.u0 : (k == 1 ? p.u1 : (k == 2 ? p.u2 : p.u3));
}

// Dimensionless extinction coefficients for a direction with cos(theta') =
// ct to the grain axis (dipole: cross sections from Im of the
// polarizability, normalised by the orientation average).
template <typename R, bool SPHERE>
__device__ __forceinline__ void alphas(const DustDev& D, R ct, R& a1, R& a2, R& a3) {
  if (SPHERE) { a1 = (R)1; a2 = (R)0; a3 = (R)0; return; }
  R cth = (R)D.ap_im * ct * ct + (R)D.aa_im * (sizeof(R) == 4 ? ((R)1 - ct) * ((R)1 + ct) : (R)1 - ct * ct);
  R cph = (R)D.ap_im;
  a1 = (cth + cph) * (R)D.inv2cavg;
  a2 = (cth - cph) * (R)D.inv2cavg;
  a3 = (R)D.alpha3_scale * a2;
}

// Isotropic direction from two uniforms: mu = 2 u0 - 1, azimuth 2 pi u1.
template <typename R>
__device__ __forceinline__ void isotropic_dir(Packet<R>& p, double u0, double u1) {
  const double mu = 2.0 * u0 - 1.0;
  const double s = sqrt(fmax(0.0, 1.0 - mu * mu));
  double sp, cp;
  sincospi(2.0 * u1, &sp, &cp);
  p.nx = s * cp; p.ny = s * sp; p.nz = mu;
}

// The cell emitting a packet of the dust's thermal emission: the first cell
// whose running luminosity sum exceeds u L.  The guide table brackets it:
// entry k - 1 (or cell 0) from below and entry k + 1 from above, k =
// floor(u ncell), so the search spans only the cells between two guide
// points.
__device__ __forceinline__ uint64_t emission_cell(const double* F, const uint32_t* G, uint64_t ncell,
                                                  double u) {
  const double t = u * F[ncell - 1];
  uint64_t k = (uint64_t)(u * (double)ncell);
  if (k > ncell - 1) k = ncell - 1;
  uint64_t lo = k > 0 ? (uint64_t)G[k - 1] : 0ull, hi = (uint64_t)G[k + 1];
  while (lo < hi) {
    const uint64_t mid = lo + ((hi - lo) >> 1);
    if (t < F[mid]) hi = mid; else lo = mid + 1;
  }
  return lo;
}

// Emission (Sec. 2.2).  Point sources: isotropic direction (or the pencil
// direction), an unpolarised Stokes vector of weight lum/N, and the cell
// holding the source (a coordinate on a face belongs to the cell the
// direction points into).  Thermal emission of the dust (the alpha_abs B
// term of eq. polarized-rt): the cell drawn by luminosity 4 pi rho kappa_abs
// B V, the position uniform in it, an isotropic direction and the Stokes
// vector w (alpha1, alpha2, 0, 0) in the grain-frame basis of the direction
// (the dichroism of absorption is that of extinction), carried to the lab
// basis; its mean over directions is w.  Draws: cell, three coordinates,
// two for the direction.  Then an exponential scattering depth.  Returns
// false if a point source lies outside the grid.
// ---------------------------------------------------------------------------
// Composite mesh with static refinement (Sec. 2: the mesh the packets
// cross).  Inside a leaf block the cell walk is the uniform one; leaving it,
// the point is expressed in finest-cell units (exact on the crossed face,
// since cell edges are powers of two of the finest one), its finest cell
// taken with the face rule (a coordinate on a face belongs to the cell the
// direction points into), and the leaf holding that cell found by
// descending from its root block.
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long finest_cell(double t, double n) {
  const double fl = floor(t);
  long long X = (long long)fl;
  if (fl == t && n < 0.0) X -= 1;
  return X;
}

__device__ __forceinline__ int mesh_find(const MeshDev& m, const long long X[3]) {
  const long long full = (long long)m.block << m.max_level;
  const long long r0 = X[0] / full, r1 = X[1] / full, r2 = X[2] / full;
  int node = (int)(r0 + (long long)m.rx * (r1 + (long long)m.ry * r2));
  long long o0 = r0 * full, o1 = r1 * full, o2 = r2 * full, size = full;
  for (int c = m.child[node]; c >= 0; c = m.child[node]) {
    size >>= 1;
    int oct = 0;
    if (X[0] - o0 >= size) { oct |= 1; o0 += size; }
    if (X[1] - o1 >= size) { oct |= 2; o1 += size; }
    if (X[2] - o2 >= size) { oct |= 4; o2 += size; }
    node = c + oct;
  }
  return m.leaf_of_node[node];
}

// the packet at finest-unit position t in finest cell X: leaf, local cell,
// fractions, and the cell-length constants of the leaf's level
template <typename R>
__device__ __forceinline__ void mesh_place(Packet<R>& p, const TransportArgs& a, const double t[3],
                                           const long long X[3]) {
  const MeshDev& m = a.mesh;
  const int j = mesh_find(m, X);
  const int4 o = reinterpret_cast<const int4*>(m.leaf_org)[j];
  const int sh = m.max_level - o.w;
  const double s = (double)(1ll << sh);
  p.leaf = j;
  p.lvl = o.w;
  const long long i0 = (X[0] - o.x) >> sh, i1 = (X[1] - o.y) >> sh, i2 = (X[2] - o.z) >> sh;
  p.ci = (int)i0; p.cj = (int)i1; p.ck = (int)i2;
  p.fx = fmin(1.0, fmax(0.0, (t[0] - (double)o.x) / s - (double)i0));
  p.fy = fmin(1.0, fmax(0.0, (t[1] - (double)o.y) / s - (double)i1));
  p.fz = fmin(1.0, fmax(0.0, (t[2] - (double)o.z) / s - (double)i2));
  const DustDev& D = a.dust[p.lam];
  const double sc = ldexp(1.0, -o.w);
  p.ks = D.ks_cell * sc;
  p.ke = D.ke_cell * sc;
  p.ka = (R)(D.ka_cell * sc);
}

// after a face crossing moved a local index out of the leaf block: the leaf
// beyond, or true if the packet left the domain
template <typename R>
__device__ bool mesh_cross(Packet<R>& p, const TransportArgs& a) {
  const MeshDev& m = a.mesh;
  const int4 o = reinterpret_cast<const int4*>(m.leaf_org)[p.leaf];
  const double s = (double)(1ll << (m.max_level - o.w));
  const double t[3] = {(double)o.x + ((double)p.ci + p.fx) * s, (double)o.y + ((double)p.cj + p.fy) * s,
                       (double)o.z + ((double)p.ck + p.fz) * s};
  const double n[3] = {p.nx, p.ny, p.nz};
  long long X[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    X[k] = finest_cell(t[k], n[k]);
    if (X[k] < 0 || X[k] >= m.nfine[k]) return true;
  }
  mesh_place(p, a, t, X);
  return false;
}

// A ray (direction om) in leaf `leaf` at local cell ci, fraction f whose
// index on some axis left the leaf: the leaf beyond (leaf, lvl, ci, f
// updated), or false if the ray left the domain.
__device__ __forceinline__ bool mesh_ray_cross(const MeshDev& m, int& leaf, int& lvl, int ci[3], double f[3],
                                               const double om[3]) {
  const int4 o = reinterpret_cast<const int4*>(m.leaf_org)[leaf];
  const double sz = (double)(1ll << (m.max_level - o.w));
  const long long X0[3] = {o.x, o.y, o.z};
  double t[3];
  long long X[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    t[k] = (double)X0[k] + ((double)ci[k] + f[k]) * sz;
    X[k] = finest_cell(t[k], om[k]);
    if (X[k] < 0 || X[k] >= m.nfine[k]) return false;
  }
  leaf = mesh_find(m, X);
  const int4 o1 = reinterpret_cast<const int4*>(m.leaf_org)[leaf];
  lvl = o1.w;
  const int sh = m.max_level - lvl;
  const long long X1[3] = {o1.x, o1.y, o1.z};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const long long i = (X[k] - X1[k]) >> sh;
    ci[k] = (int)i;
    f[k] = fmin(1.0, fmax(0.0, (t[k] - (double)X1[k]) / (double)(1ll << sh) - (double)i));
  }
  return true;
}

// flat index of the packet's cell
template <bool MESH, typename R>
__device__ __forceinline__ uint64_t cell_index(const Packet<R>& p, const TransportArgs& a) {
  if (MESH) {
    const uint64_t B = (uint64_t)a.mesh.block;
    return (uint64_t)p.leaf * B * B * B + (uint64_t)p.ci + B * ((uint64_t)p.cj + B * (uint64_t)p.ck);
  }
  return (uint64_t)p.ci + (uint64_t)a.nx * ((uint64_t)p.cj + (uint64_t)a.ny * p.ck);
}

template <typename R, bool ALIGNED, bool SPHERE, bool MESH>
__device__ bool init_packet(Packet<R>& p, uint64_t g, const TransportArgs& a) {
  int lo = 0, hi = a.n_lambda - 1;
  while (lo < hi) {  // last wavelength whose first index <= g
    int mid = (lo + hi + 1) >> 1;
    if (a.dust[mid].first <= g) lo = mid; else hi = mid - 1;
  }
  p.lam = lo;
  p.pid = g - a.dust[lo].first;
  p.draw = 0;
  p.blk = 0xffffffffu;
  p.w0 = (R)a.dust[lo].w0;
  p.ks = a.dust[lo].ks_cell;
  p.ke = a.dust[lo].ke_cell;
  p.ka = (R)a.dust[lo].ka_cell;
  p.e_abs = 0.0; p.e_scat = 0.0; p.e_gain = 0.0;
  p.tau_path = (R)0;
  p.events = 0; p.steps = 0; p.trials = 0; p.rr = 0;
  p.hash = 14695981039346656037ull;
  p.last = -1;
  bool in = true;
  if (a.src_kind == 2) {
    const uint64_t c = emission_cell(a.em_cdf + (uint64_t)lo * a.ncell,
                                     a.em_guide + (uint64_t)lo * (a.ncell + 1), a.ncell,
                                     (double)next_uniform(p, a.seed));
    if (MESH) {
      // cell c of the mesh: leaf c / block^3, local cell x fastest; the
      // cell-length constants of the leaf's level
      const uint64_t Bm = (uint64_t)a.mesh.block, r = c % (Bm * Bm * Bm);
      p.leaf = (int)(c / (Bm * Bm * Bm));
      p.ci = (int)(r % Bm);
      p.cj = (int)((r / Bm) % Bm);
      p.ck = (int)(r / (Bm * Bm));
      p.lvl = a.mesh.leaf_org[4 * p.leaf + 3];
      const double sc = ldexp(1.0, -p.lvl);
      p.ks = a.dust[lo].ks_cell * sc;
      p.ke = a.dust[lo].ke_cell * sc;
      p.ka = (R)(a.dust[lo].ka_cell * sc);
    } else {
      p.ci = (int)(c % (uint64_t)a.nx);
      p.cj = (int)((c / (uint64_t)a.nx) % (uint64_t)a.ny);
      p.ck = (int)(c / ((uint64_t)a.nx * (uint64_t)a.ny));
    }
    p.fx = (double)next_uniform(p, a.seed);
    p.fy = (double)next_uniform(p, a.seed);
    p.fz = (double)next_uniform(p, a.seed);
    const double u0 = (double)next_uniform(p, a.seed), u1 = (double)next_uniform(p, a.seed);
    isotropic_dir(p, u0, u1);
    const double w = a.dust[lo].w0;
    if (SPHERE) {
      p.I = (R)w; p.Q = (R)0; p.U = (R)0; p.V = (R)0;
    } else {
      const V3<double> nd{p.nx, p.ny, p.nz};
      V3<double> ngd = nd;
      double c2 = 1.0, s2 = 0.0;
      if (ALIGNED) {
        const Quat<double> qd = grain_quat(V3<double>{(double)a.bx[c], (double)a.by[c], (double)a.bz[c]});
        ngd = to_grain(qd, nd);
        eta2(qd, nd, ngd, c2, s2);
      }
      double a1, a2, a3;
      alphas<double, SPHERE>(a.dust[lo], ngd.z, a1, a2, a3);
      p.I = (R)(w * a1); p.Q = (R)(c2 * w * a2); p.U = (R)(s2 * w * a2); p.V = (R)0;
    }
    p.rho = a.rho[c];
  } else {
    const double u0 = (double)next_uniform(p, a.seed), u1 = (double)next_uniform(p, a.seed);
    if (a.src_kind == 1) {
      p.nx = a.dx_; p.ny = a.dy_; p.nz = a.dz_;
    } else {
      isotropic_dir(p, u0, u1);
    }
    p.I = p.w0; p.Q = (R)0; p.U = (R)0; p.V = (R)0;
    const double pos[3] = {a.sx, a.sy, a.sz}, org[3] = {a.x0, a.y0, a.z0};
    const double dir[3] = {p.nx, p.ny, p.nz};
    if (MESH) {
      // the finest cell holding the source (face rule), then its leaf
      double t[3];
      long long X[3];
      in = true;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        t[k] = (pos[k] - org[k]) / a.mesh.fine;
        X[k] = finest_cell(t[k], dir[k]);
        in = in && X[k] >= 0 && X[k] < a.mesh.nfine[k];
      }
      if (in) mesh_place(p, a, t, X);
      p.rho = in ? a.rho[cell_index<true>(p, a)] : 0.f;
      p.rnx = 1.0 / p.nx; p.rny = 1.0 / p.ny; p.rnz = 1.0 / p.nz;
      p.tau = -log((double)next_uniform(p, a.seed));
      return in;
    }
    int ci[3];
    double fr[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double t = (pos[k] - org[k]) / a.dx;
      double fl = floor(t);
      double f = t - fl;
      int i = (int)fl;
      if (f == 0.0 && dir[k] < 0.0) { i -= 1; f = 1.0; }
      ci[k] = i;
      fr[k] = f;
    }
    const int nn[3] = {a.nx, a.ny, a.nz};
#pragma unroll
    for (int k = 0; k < 3; ++k)  // a periodic axis holds every coordinate
      if ((a.boundary >> k) & 1) ci[k] = ((ci[k] % nn[k]) + nn[k]) % nn[k];
    p.ci = ci[0]; p.cj = ci[1]; p.ck = ci[2];
    p.fx = fr[0]; p.fy = fr[1]; p.fz = fr[2];
    in = p.ci >= 0 && p.ci < a.nx && p.cj >= 0 && p.cj < a.ny && p.ck >= 0 && p.ck < a.nz;
    p.rho = in ? a.rho[(uint64_t)p.ci + (uint64_t)a.nx * ((uint64_t)p.cj + (uint64_t)a.ny * p.ck)] : 0.f;
  }
  p.rnx = 1.0 / p.nx; p.rny = 1.0 / p.ny; p.rnz = 1.0 / p.nz;
  p.tau = -log((double)next_uniform(p, a.seed));
  return in;
}

// Coherency contribution of a segment-integrated Stokes vector J (lab basis of
// n): sum_ab rho_ab e_a e_b^T with rho = 1/2 [[I+Q, U-iV],[U+iV, I-Q]],
// e1 = theta_hat(n), e2 = phi_hat(n), times the weight w.  Output order: real
// xx yy zz xy xz yz, imaginary yz zx xy (the antisymmetric part equals
// -V/2 [n]_x in this basis).
// With e1 = (nz cos p, nz sin p, -sin t), e2 = (-sin p, cos p, 0) every
// product of two basis components is written with cos^2 p, sin^2 p,
// cos p sin p (from n by one reciprocal of nx^2 + ny^2) and sin t cos p = nx,
// sin t sin p = ny: no square root per step.  At the pole (phi = 0) cos p = 1
// and sin t = sqrt(nx^2 + ny^2).
template <typename R, int NC>
__device__ __forceinline__ void coherency(const V3<R>& n, R JI, R JQ, R JU, R JV, R w,
                                          R out[NC]) {
  const R r2 = n.x * n.x + n.y * n.y;
  R px, py, cc, ss, cs;  // sin t cos p, sin t sin p, cos^2 p, sin^2 p, cos p sin p
  if (r2 <= (R)KP_POLE2) {
    px = k_sqrt(r2); py = (R)0; cc = (R)1; ss = (R)0; cs = (R)0;
  } else {
    const R ir = (R)1 / r2;
    px = n.x; py = n.y; cc = n.x * n.x * ir; ss = n.y * n.y * ir; cs = n.x * n.y * ir;
  }
  R a = (R)0.5 * (JI + JQ) * w, b = (R)0.5 * (JI - JQ) * w, u = (R)0.5 * JU * w;
  R v = (R)-0.5 * JV * w;
  const R an2 = a * n.z * n.z, un = u * n.z;
  out[0] = an2 * cc + b * ss - (R)2 * un * cs;
  out[1] = an2 * ss + b * cc + (R)2 * un * cs;
  out[2] = a * r2;
  out[3] = (an2 - b) * cs + un * (cc - ss);
  out[4] = -a * n.z * px + u * py;
  out[5] = -a * n.z * py - u * px;
  if (NC > 6) {
    out[NC > 6 ? 6 : 0] = v * n.x;
    out[NC > 7 ? 7 : 0] = v * n.y;
    out[NC > 8 ? 8 : 0] = v * n.z;
  }
}

// Components of the tally kept per cell and the per-cell stride in doubles:
// spheres never create circular polarisation from unpolarised light, so the
// antisymmetric (V) part of the coherency is identically zero.
// Per-cell tally block of TS doubles (one 64- or 128-byte aligned block):
// slots [0, NC) the coherency sums.  For non-spherical grains slot NC holds
// the cell's density and slots NC+1..NC+4 the unit quaternion (w, x, y, z) of
// its grain frame, formed once per run from the alignment direction (eq.
// grain-quaternion) instead of at every step and scattering: the step that
// enters a cell reads them from the block whose coherency it adds to when it
// leaves, one 128-byte line instead of four (density and three direction
// planes, 256 MB at 256^3, too large to stay in the Infinity Cache).  Spherical grains read the density from the compact FP32 array
// (64 MB at 256^3), which stays cache-resident; there the density load is
// the step's critical-path latency and the tally line's fetch is better
// left to the atomics, off that path.
template <bool SPHERE> struct TallyShape {
  static constexpr int NC = SPHERE ? 6 : 9;
  static constexpr int TS = SPHERE ? 8 : 16;
  static constexpr int RHO = NC;
  static constexpr bool HAS_B = !SPHERE;  // density and grain quaternion in slots NC..NC+4
};

// The grain-frame quaternion of a cell: from its tally block, or formed from
// the alignment direction when the block does not hold it.
template <bool ALIGNED, bool SPHERE>
__device__ __forceinline__ Quat<double> cell_quat(const TransportArgs& a, const double* blk, uint64_t c) {
  using TSh = TallyShape<SPHERE>;
  if (TSh::HAS_B) return Quat<double>{blk[TSh::RHO + 1], blk[TSh::RHO + 2], blk[TSh::RHO + 3], blk[TSh::RHO + 4]};
  return grain_quat(V3<double>{(double)a.bx[c], (double)a.by[c], (double)a.bz[c]});
}

template <typename R>
__device__ __forceinline__ Quat<R> quat_cast(const Quat<double>& q) {
  return Quat<R>{(R)q.w, (R)q.x, (R)q.y, (R)q.z};
}

// Tally flush, wave-cooperative and deferred.  A lane that leaves a cell
// stages (key, NC values) in its wavefront's LDS area (wave_stage); when the
// area may not hold another full wavefront of entries, wave_drain adds all
// staged entries to the tally: lane L adds component L % NC of entry L / NC,
// so one atomic instruction covers 64 / NC whole cells.  Deferring matters on
// gfx9: atomics without return still count in vmcnt, and the next density
// load's wait (vmcnt(0)) would otherwise wait every iteration for the last
// flush's read-modify-writes to reach memory; drained every few iterations,
// that latency is exposed once per drain.  Both must be reached by all lanes
// of the wavefront; `staged` is the same in every lane.
template <int NC>
__device__ __forceinline__ int wave_stage(bool need, int64_t key, const double acc[NC], double* sv, long long* sk,
                                          int lane, int& staged) {
  const unsigned long long mask = __ballot(need);
  if (mask == 0ull) return 0;
  if (need) {
    const int r = staged + __popcll(mask & ((1ull << lane) - 1ull));
#pragma unroll
    for (int k = 0; k < NC; ++k) sv[r * NC + k] = acc[k];
    sk[r] = key;
  }
  const int n = __popcll(mask);
  staged += n;
  return n;
}

template <int NC, int TS>
__device__ __forceinline__ void wave_drain(double* tally, double* sv, long long* sk, int lane, int& staged) {
  const int n = staged;
  if (n == 0) return;
  staged = 0;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  constexpr int G = 64 / NC;
  constexpr int U = 4;  // rounds whose LDS reads are issued before one wait
  const int slot = lane / NC, k = lane - slot * NC;
  if (slot < G) {
    for (int base = 0; base < n; base += U * G) {
      double v[U];
      long long key_r[U];
      // reads of entries beyond n stay inside the staged entries (index
      // clamped to n - 1) and their atomics are masked below
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = min(base + u * G + slot, n - 1);
        v[u] = sv[e * NC + k];
        key_r[u] = sk[e];
      }
      // keep every key read ahead of the branches below (one LDS wait
      // for all of them instead of one per round)
#pragma unroll
      for (int u = 0; u < U; ++u) asm volatile("" : : "v"(key_r[u]));
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (base + u * G + slot < n && v[u] != 0.0)
          unsafeAtomicAdd(tally + (uint64_t)key_r[u] * TS + k, v[u]);
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Scattering event (Sec. 2.2; rejection sampling of Sec. 3): incident state
// carried into the grain frame, proposals uniform on the sphere there
// (cos, azimuth, acceptance: three uniforms per trial), accepted when
// u * bound <= [P s]_I, output rescaled to the scattered power, then carried
// back to the lab frame.  Returns false on a numerical failure.
template <typename R, bool ALIGNED, bool SPHERE>
__device__ bool scatter(Packet<R>& p, const Quat<R>& q, const Quat<double>& qd,
                        const DustDev& D, uint64_t seed) {
  const V3<R> n{(R)p.nx, (R)p.ny, (R)p.nz};
  V3<R> ng = n;
  R c2 = (R)1, s2 = (R)0;
  R cpn, spn, stn;
  if (ALIGNED) {
    // The grain-frame direction and its azimuth are formed in FP64: for a
    // packet moving nearly along the grain axis the transverse components
    // are small differences of order-one terms, which FP32 resolves only to
    // ~1e-7 absolute, i.e. to a basis angle error of ~1e-7 / sin(theta').
    const V3<double> nd{p.nx, p.ny, p.nz};
    const V3<double> ngd = to_grain(qd, nd);
    double cpd, spd, std_;
    azimuth(ngd, cpd, spd, std_);
    ng = V3<R>{(R)ngd.x, (R)ngd.y, (R)ngd.z};
    cpn = (R)cpd;
    spn = (R)spd;
    stn = (R)std_;
    eta2(q, n, ng, c2, s2);
  } else {
    azimuth(ng, cpn, spn, stn);
  }
  const R I = p.I, Qg = c2 * p.Q + s2 * p.U, Ug = -s2 * p.Q + c2 * p.U, V = p.V;
  V3<R> e1, e2;
  e1 = {ng.z * cpn, ng.z * spn, -stn};
  e2 = {-spn, cpn, (R)0};
  const R r11 = (R)0.5 * (I + Qg), r22 = (R)0.5 * (I - Qg);
  const Cx<R> r12{(R)0.5 * Ug, (R)-0.5 * V};
  const R pf = (R)D.pfac;
  const R bound = (R)D.bound_fac * I;
  const R tol = sizeof(R) == 4 ? (R)1e-4 : (R)1e-12;
  const Cx<R> ap{(R)D.ap_re, (R)D.ap_im};
  const Cx<R> dd{(R)(D.aa_re - D.ap_re), (R)(D.aa_im - D.ap_im)};
  Cx<R> J11, J12, J21, J22;
  R mu = 0, smu = 0, cph = 1, sph = 0, Iout = 0, umu = 0, uph = 0;
  bool ok = false;
  for (int trial = 0; trial < 100000; ++trial) {
    umu = next_uniform(p, seed);
    mu = (R)2 * umu - (R)1;
    uph = next_uniform(p, seed);
    R ua = next_uniform(p, seed);
    p.trials++;
    // 1 - mu^2 as (1 - mu)(1 + mu): both factors are exact, so sin theta'
    // keeps full relative precision near the grain axis in FP32
    smu = sizeof(R) == 4 ? k_sqrt(fmax((R)0, ((R)1 - mu) * ((R)1 + mu))) : k_sqrt(fmax((R)0, (R)1 - mu * mu));
    k_sincospi((R)2 * uph, &sph, &cph);
    if (smu * smu <= (R)KP_POLE2) { cph = (R)1; sph = (R)0; }
    const V3<R> f1{mu * cph, mu * sph, -smu}, f2{-sph, cph, (R)0};
    const R D11 = dot(f1, e1), D12 = dot(f1, e2), D21 = dot(f2, e1), D22 = dot(f2, e2);
    if (SPHERE) {
      J11 = {D11, 0}; J12 = {D12, 0}; J21 = {D21, 0}; J22 = {D22, 0};
      Iout = pf * ((D11 * D11 + D21 * D21) * r11 + (D12 * D12 + D22 * D22) * r22 +
                   (R)2 * (D11 * D12 + D21 * D22) * r12.re);
    } else {
      J11 = cadd(cscale(ap, D11), cscale(dd, smu * stn));
      J12 = cscale(ap, D12);
      J21 = cscale(ap, D21);
      J22 = cscale(ap, D22);
      Iout = pf * (cabs2(J11) * r11 + cabs2(J12) * r22 + (R)2 * cmulc(cmul(J11, r12), J12).re +
                   cabs2(J21) * r11 + cabs2(J22) * r22 + (R)2 * cmulc(cmul(J21, r12), J22).re);
    }
    if (!(Iout <= bound * ((R)1 + tol))) return false;
    if (ua * bound <= Iout) { ok = true; break; }
  }
  if (!ok) return false;
  // full scattered state rho' = J rho J^dagger in the natural basis of mg
  const Cx<R> r21{r12.re, -r12.im};
  const Cx<R> T11 = cadd(cscale(J11, r11), cmul(J12, r21));
  const Cx<R> T12 = cadd(cmul(J11, r12), cscale(J12, r22));
  const Cx<R> T21 = cadd(cscale(J21, r11), cmul(J22, r21));
  const Cx<R> T22 = cadd(cmul(J21, r12), cscale(J22, r22));
  const R p11 = cmulc(T11, J11).re + cmulc(T12, J12).re;
  const R p22 = cmulc(T21, J21).re + cmulc(T22, J22).re;
  const Cx<R> p12 = cadd(cmulc(T11, J21), cmulc(T12, J22));
  R So = pf * (p11 + p22), Qo = pf * (p11 - p22), Uo = pf * (R)2 * p12.re,
    Vo = pf * (R)-2 * p12.im;
  // scattered power: sum_k |a_k|^2 C_kk / N_P with C_zz = r11 sin^2(theta'_n)
  R sig = I;
  if (!SPHERE) {
    R czz = r11 * stn * stn;
    sig = (R)D.ap2_np * (I - czz) + (R)D.aa2_np * czz;
  }
  R scale = sig / So;
  So = sig; Qo *= scale; Uo *= scale; Vo *= scale;
  if (sizeof(R) == 4) {
    // In FP32 the scattered state of a direction of near-zero scattered
    // intensity is a difference of terms of size I, so rounding can leave it
    // outside |P| <= I (one packet of 1.5e8 on a 256^3 disk: |P| = 1.0008 I,
    // after which the next event's bound check fails); it is projected back
    // onto the cone.
    const R p2 = Qo * Qo + Uo * Uo + Vo * Vo;
    if (p2 > So * So) {
      const R f = So / k_sqrt(p2);
      Qo *= f; Uo *= f; Vo *= f;
    }
  }
  // the accepted direction itself is formed in FP64 from the same uniforms
  const double mud = 2.0 * (double)umu - 1.0;
  const double smud = sqrt(fmax(0.0, 1.0 - mud * mud));
  double sphd, cphd;
  sincospi(2.0 * (double)uph, &sphd, &cphd);
  if (smud * smud <= KP_POLE2) { cphd = 1.0; sphd = 0.0; }
  const V3<double> mgd{smud * cphd, smud * sphd, mud};
  V3<double> md = mgd;
  R cm = (R)1, sm = (R)0;
  if (ALIGNED) {
    md = from_grain(qd, mgd);
    eta2(q, V3<R>{(R)md.x, (R)md.y, (R)md.z}, V3<R>{(R)mgd.x, (R)mgd.y, (R)mgd.z}, cm, sm);
  }
  p.nx = md.x; p.ny = md.y; p.nz = md.z;
  p.rnx = 1.0 / p.nx; p.rny = 1.0 / p.ny; p.rnz = 1.0 / p.nz;
  p.e_scat += (double)(sig - I);
  p.I = So;
  p.Q = cm * Qo - sm * Uo;
  p.U = sm * Qo + cm * Uo;
  p.V = Vo;
  return true;
}

// ---------------------------------------------------------------------------
// Tabulated scattering (Sec. 2.2: optical properties given as interpolation
// tables).  The table holds the scattering-plane elements S11 S12 S22 S33
// S34 S44 of randomly oriented grains, normalised so that S11 integrates to 1
// over solid angle, at scattering angles uniform on [0, pi]; values are linear
// in cos Theta between nodes.  FP64 throughout.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void tab_eval(const DustDev& D, double mu, double z[6]) {
  const int n = D.tab_n;
  mu = fmin(1.0, fmax(-1.0, mu));
  // the node interval: the guide's entry for the cos Theta bin (no inverse
  // cosine on the dependency chain), then forward to the interval holding mu
  const int G = D.tab_g;
  int b = (int)((1.0 - mu) * (0.5 * (double)G));
  b = b < 0 ? 0 : (b > G - 1 ? G - 1 : b);
  int j = D.tab_guide[b];
  const double* M = D.tab_mu;
  while (j < n - 2 && mu < M[j + 1]) ++j;
  while (j > 0 && mu > M[j]) --j;
  const double ma = M[j], mb = M[j + 1];
  const double t = ma > mb ? (ma - mu) / (ma - mb) : 0.0;
  const double* Z = D.tab + 6 * j;
#pragma unroll
  for (int k = 0; k < 6; ++k) z[k] = (1.0 - t) * Z[k] + t * Z[6 + k];
}

// P(m; n) s per unit solid angle: s in the lab basis of n, the result in the
// basis (tm, pm) of m.  The scattering plane's normal is e = n x m / |n x m|
// (phi_hat of n when m = +-n); with a = m . theta_hat_n, b = m . phi_hat_n
// (|n x m|^2 = a^2 + b^2) the rotation into the plane basis (e x n, e) is
// cos 2psi = (a^2 - b^2) / |n x m|^2, sin 2psi = 2ab / |n x m|^2, and the
// rotation out of (e x m, e) into (tm, pm) is by -chi with
// cos 2chi = ((n.tm)^2 - (n.pm)^2) / |n x m|^2, sin 2chi = 2 (n.tm)(n.pm) /
// |n x m|^2: no square root or angle is formed.
__device__ __forceinline__ void tab_toward(const DustDev& D, const V3<double>& n, const double s[4],
                                           const V3<double>& m, const V3<double>& tm,
                                           const V3<double>& pm, double out[4]) {
  V3<double> thn, phn;
  basis(n, thn, phn);
  const double a = dot(m, thn), b = dot(m, phn);
  const double w2 = a * a + b * b;
  double c2p = 1.0, s2p = 0.0, c2c, s2c;
  if (w2 > 1e-24) {
    const double iw = 1.0 / w2;
    c2p = (a * a - b * b) * iw;
    s2p = 2.0 * a * b * iw;
    const double ct = dot(n, tm), cp = dot(n, pm);
    c2c = (ct * ct - cp * cp) * iw;
    s2c = 2.0 * ct * cp * iw;
  } else {
    const double cc = dot(phn, pm), ss = -dot(phn, tm);
    c2c = cc * cc - ss * ss;
    s2c = 2.0 * cc * ss;
  }
  const double Qp = c2p * s[1] + s2p * s[2], Up = -s2p * s[1] + c2p * s[2];
  double z[6];
  tab_eval(D, dot(n, m), z);
  const double I = z[0] * s[0] + z[1] * Qp, Q = z[1] * s[0] + z[2] * Qp;
  const double U = z[3] * Up + z[4] * s[3], V = -z[4] * Up + z[5] * s[3];
  out[0] = I;
  out[1] = c2c * Q - s2c * U;
  out[2] = s2c * Q + c2c * U;
  out[3] = V;
}

// Scattering event of tabulated grains: envelope rejection.  Per trial four
// uniforms: the node interval by the envelope's cumulative mass (the larger
// S11 of its two nodes times the interval's width in cos Theta), cos Theta
// uniform inside it, the azimuth, and acceptance of u * max S11 (I + |P_lin|)
// <= the scattered I.  The total scattered power does not depend on the
// polarisation, so the scattered state is rescaled to the incident I.
template <typename R>
__device__ bool scatter_tab(Packet<R>& p, const DustDev& D, uint64_t seed) {
  const V3<double> n{p.nx, p.ny, p.nz};
  V3<double> th, ph;
  basis(n, th, ph);
  const double s[4] = {(double)p.I, (double)p.Q, (double)p.U, (double)p.V};
  const double plin = sqrt(s[1] * s[1] + s[2] * s[2]);
  const int nt = D.tab_n;
  const double* cum = D.tab_cum;
  const double total = cum[nt - 1];
  for (int trial = 0; trial < 100000; ++trial) {
    const double u1 = (double)next_uniform(p, seed), u2 = (double)next_uniform(p, seed);
    const double u3 = (double)next_uniform(p, seed), u4 = (double)next_uniform(p, seed);
    p.trials++;
    // the first interval whose cumulative envelope mass exceeds u1 * total
    const double target = u1 * total;
    int lo = 0, hi = nt - 2;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (cum[mid + 1] > target) hi = mid;
      else lo = mid + 1;
    }
    const int j = lo;
    const double ma = D.tab_mu[j], mb = D.tab_mu[j + 1];
    const double mu = ma + u2 * (mb - ma);
    double sp, cp;
    sincospi(2.0 * u3, &sp, &cp);
    const double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    V3<double> m{mu * n.x + st * (cp * th.x + sp * ph.x), mu * n.y + st * (cp * th.y + sp * ph.y),
                 mu * n.z + st * (cp * th.z + sp * ph.z)};
    const double inm = 1.0 / sqrt(dot(m, m));
    m = V3<double>{m.x * inm, m.y * inm, m.z * inm};
    V3<double> tm, pm;
    basis(m, tm, pm);
    double o[4];
    tab_toward(D, n, s, m, tm, pm, o);
    const double env = fmax(D.tab[6 * j], D.tab[6 * (j + 1)]) * (s[0] + plin);
    if (!(o[0] <= env * (1.0 + 1e-9))) return false;
    if (u4 * env <= o[0]) {
      const double scale = s[0] / o[0];
      p.nx = m.x; p.ny = m.y; p.nz = m.z;
      p.rnx = 1.0 / p.nx; p.rny = 1.0 / p.ny; p.rnz = 1.0 / p.nz;
      const R Io = (R)(o[0] * scale);
      p.e_scat += (double)(Io - p.I);
      p.I = Io;
      p.Q = (R)(o[1] * scale);
      p.U = (R)(o[2] * scale);
      p.V = (R)(o[3] * scale);
      return true;
    }
  }
  return false;
}

template <bool MESH, typename R>
__device__ uint32_t roulette(Packet<R>& p, const TransportArgs& a);

// One loop iteration: one cell segment (Sec. 2.2: cell-to-cell traversal,
// exponential scattering depth, continuous extinction across the segment by
// the analytic cell solution of Appendix A, tally of the segment into the
// scattering source of Sec. 2.3), then a scattering event or the crossing
// into the next cell, then Russian roulette.  Returns 0 or an end kind.
template <typename R, bool ALIGNED, bool SPHERE, bool TAB, bool MESH>
__device__ uint32_t step(Packet<R>& p, const TransportArgs& a, bool& has, int64_t& key,
                         R cc[TallyShape<SPHERE>::NC], bool& pending) {
  constexpr int NC = TallyShape<SPHERE>::NC;
  static_assert(!TAB || (SPHERE && !ALIGNED), "tabulated grains have scalar extinction");
  const uint64_t c = cell_index<MESH>(p, a);
  p.last = (int64_t)c;
  if (p.events >= a.max_events || p.steps >= KP_MAX_STEPS) {
    p.hash = hash_event(p.hash, END_BUDGET, c);
    return END_BUDGET;
  }
  const double inf = __builtin_huge_val();
  const double dnx = p.nx, dny = p.ny, dnz = p.nz;
  // distances to the exit faces (reciprocals of n formed when n changes)
  double tx = dnx > 0.0 ? (1.0 - p.fx) * p.rnx : (dnx < 0.0 ? -p.fx * p.rnx : inf);
  double ty = dny > 0.0 ? (1.0 - p.fy) * p.rny : (dny < 0.0 ? -p.fy * p.rny : inf);
  double tz = dnz > 0.0 ? (1.0 - p.fz) * p.rnz : (dnz < 0.0 ? -p.fz * p.rnz : inf);
  double td = tx;
  int axis = 0;
  if (ty < td) { td = ty; axis = 1; }
  if (tz < td) { td = tz; axis = 2; }
  if (!(td < inf)) return END_NUMERIC;
  const DustDev& D = a.dust[p.lam];
  const uint64_t sl = tally_slot(c, p.ci, p.cj, p.ck, MESH ? 0 : a.tbx, a.tby);
  const double* blk = a.tally + ((uint64_t)p.lam * a.nslot + sl) * TallyShape<SPHERE>::TS;
  const double rhod = TallyShape<SPHERE>::HAS_B ? blk[TallyShape<SPHERE>::RHO] : (double)p.rho;
  const double kbd = rhod * p.ks;
  double tld;
  bool scat;
  if (kbd > 0.0 && p.tau < kbd * td) { tld = p.tau / kbd; scat = true; }
  else { tld = td; p.tau -= kbd * td; scat = false; }
  const R rho = (R)rhod, kb = (R)kbd, tl = (R)tld;
  p.steps++;
  Quat<R> q{(R)1, (R)0, (R)0, (R)0};
  Quat<double> qd{1.0, 0.0, 0.0, 0.0};
  if (ALIGNED && rho > (R)0) {
    qd = cell_quat<ALIGNED, SPHERE>(a, blk, c);
    q = quat_cast<R>(qd);
  }
  if (rho > (R)0 && tl > (R)0) {
    const V3<R> n{(R)p.nx, (R)p.ny, (R)p.nz};
    const R Ib = p.I;
    R JI, JQ, JU, JV;
    if (SPHERE && !ALIGNED) {
      // spheres: extinction is the scalar absorption e^{-rho kappa_abs l}
      const R m1 = rho * p.ka;
      const R E = k_exp(-m1 * tl), G = tl * phi1(m1 * tl);
      p.tau_path += m1 * tl;
      JI = p.I * G; JQ = p.Q * G; JU = p.U * G; JV = p.V * G;
      p.I *= E; p.Q *= E; p.U *= E; p.V *= E;
    } else {
      // The exponents are differences of two cell-scale optical depths
      // (rho kappa_ext alpha vs rho kappa_sca, each up to ~1e3 per cell), so
      // the grain-frame direction, the alphas and the exponents are formed in
      // FP64; the exponentials and the Stokes arithmetic run in R.
      const V3<double> nd{p.nx, p.ny, p.nz};
      V3<double> ngd = nd;
      if (ALIGNED) ngd = to_grain(qd, nd);
      R c2 = (R)1, s2 = (R)0;
      if (ALIGNED) eta2(q, n, V3<R>{(R)ngd.x, (R)ngd.y, (R)ngd.z}, c2, s2);
      double a1, a2, a3;
      alphas<double, SPHERE>(D, ngd.z, a1, a2, a3);
      const double ked = rhod * p.ke;
      const double xAd = (ked * (a1 + a2) - kbd) * tld, xBd = (ked * (a1 - a2) - kbd) * tld;
      const double xUd = (ked * a1 - kbd) * tld, yd = ked * a3 * tld;
      const R xA = (R)xAd, xB = (R)xBd, xU = (R)xUd;
      p.tau_path += (R)fabs(xUd);
      const R Qg = c2 * p.Q + s2 * p.U, Ug = -s2 * p.Q + c2 * p.U;
      const R A = p.I + Qg, B = p.I - Qg;
      const R gA = tl * phi1(xA), gB = tl * phi1(xB);
      const R eA = k_exp(-xA), eB = k_exp(-xB);
      R JUg, JVg, Un, Vn;
      if (yd == 0.0) {
        const R gU = tl * phi1(xU), eU = k_exp(-xU);
        JUg = Ug * gU; JVg = p.V * gU;
        Un = Ug * eU; Vn = p.V * eU;
      } else {
        // U + iV evolves as exp((-mU + i w) s)
        const R x = -xU, y = (R)yd;
        const R ex = k_exp(x), cy = k_cos(y), sy = k_sin(y), sh = k_sin((R)0.5 * y);
        const Cx<R> ez{ex * cy, ex * sy};
        const Cx<R> em1{k_expm1(x) * cy - (R)2 * sh * sh, ex * sy};
        const R den = x * x + y * y;
        const Cx<R> phic{(em1.re * x + em1.im * y) / den, (em1.im * x - em1.re * y) / den};
        const Cx<R> Z{Ug, p.V};
        const Cx<R> JZ = cscale(cmul(Z, phic), tl), Zn = cmul(Z, ez);
        JUg = JZ.re; JVg = JZ.im; Un = Zn.re; Vn = Zn.im;
      }
      const R JA = A * gA, JB = B * gB, An = A * eA, Bn = B * eB;
      const R JQg = (R)0.5 * (JA - JB), Qn = (R)0.5 * (An - Bn);
      JI = (R)0.5 * (JA + JB);
      JQ = c2 * JQg - s2 * JUg;
      JU = s2 * JQg + c2 * JUg;
      JV = JVg;
      p.I = (R)0.5 * (An + Bn);
      p.Q = c2 * Qn - s2 * Un;
      p.U = s2 * Qn + c2 * Un;
      p.V = Vn;
    }
    p.e_abs += (double)(Ib - p.I);
    if (kb > (R)0) {
      if (TAB) {
        // tabulated grains: the segment's Stokes integral itself (in the lab
        // basis of n), projected on every camera when it is flushed
        cc[0] = JI * kb; cc[1] = JQ * kb; cc[2] = JU * kb; cc[3] = JV * kb;
      } else {
        coherency<R, NC>(n, JI, JQ, JU, JV, kb, cc);
      }
      key = (int64_t)((uint64_t)p.lam * a.nslot + sl);
      has = true;
    }
  }
  if (!(p.I > (R)0)) {
    // the weight underflowed in a very thick absorbing segment: the packet is
    // absorbed (a non-finite weight is reported as a numerical failure)
    if (!isfinite(p.I)) return END_NUMERIC;
    p.hash = hash_event(p.hash, END_RR_KILL, c);
    return END_RR_KILL;
  }
  if (scat) {
    // the scattering event itself runs in scatter_step(), possibly a few
    // iterations later together with other lanes of the wavefront
    p.fx = fmin(1.0, fmax(0.0, p.fx + tld * dnx));
    p.fy = fmin(1.0, fmax(0.0, p.fy + tld * dny));
    p.fz = fmin(1.0, fmax(0.0, p.fz + tld * dnz));
    pending = true;
    return 0;
  } else {
    if (axis != 0) p.fx = fmin(1.0, fmax(0.0, p.fx + td * dnx));
    if (axis != 1) p.fy = fmin(1.0, fmax(0.0, p.fy + td * dny));
    if (axis != 2) p.fz = fmin(1.0, fmax(0.0, p.fz + td * dnz));
    bool out;
    // leaving through an open face ends the packet; a periodic face brings
    // it back through the opposite one; on a mesh, leaving the leaf block
    // moves it into the leaf beyond
    const int nbx = MESH ? a.mesh.block : a.nx, nby = MESH ? a.mesh.block : a.ny;
    const int nbz = MESH ? a.mesh.block : a.nz;
    if (axis == 0) {
      if (dnx > 0.0) { p.ci++; p.fx = 0.0; } else { p.ci--; p.fx = 1.0; }
      out = p.ci < 0 || p.ci >= nbx;
    } else if (axis == 1) {
      if (dny > 0.0) { p.cj++; p.fy = 0.0; } else { p.cj--; p.fy = 1.0; }
      out = p.cj < 0 || p.cj >= nby;
    } else {
      if (dnz > 0.0) { p.ck++; p.fz = 0.0; } else { p.ck--; p.fz = 1.0; }
      out = p.ck < 0 || p.ck >= nbz;
    }
    // the boundary mask is the same for every lane: open grids skip the wrap
    if (!MESH && a.boundary != 0 && out && ((a.boundary >> axis) & 1)) {
      if (axis == 0) p.ci = p.ci < 0 ? a.nx - 1 : 0;
      else if (axis == 1) p.cj = p.cj < 0 ? a.ny - 1 : 0;
      else p.ck = p.ck < 0 ? a.nz - 1 : 0;
      out = false;
    }
    if (MESH && out) out = mesh_cross(p, a);
    if (out) {
      p.hash = hash_event(p.hash, END_ESCAPE, c);
      return END_ESCAPE;
    }
    // the next step's density, in flight while this iteration finishes
    if (!TallyShape<SPHERE>::HAS_B) p.rho = a.rho[cell_index<MESH>(p, a)];
  }
  return roulette<MESH>(p, a);
}

// ---------------------------------------------------------------------------
// Shared by step 2 and peel-off: the Appendix A solution in its eigenbasis
// and the Stokes source toward a camera formed from an incident coherency.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void appA_eigen(double a1, double a2, double a3, double dtau,
                                           const double src[4], double s[4]) {
  const double a = a1 + a2, b = a1 - a2;
  const double A = s[0] + s[1], B = s[0] - s[1];
  const double SA = src[0] + src[1], SB = src[0] - src[1];
  const double An = A * exp(-a * dtau) + SA * dtau * phi1(a * dtau);
  const double Bn = B * exp(-b * dtau) + SB * dtau * phi1(b * dtau);
  double Un, Vn;
  if (a3 == 0.0) {
    const double e = exp(-a1 * dtau), g = dtau * phi1(a1 * dtau);
    Un = s[2] * e + src[2] * g;
    Vn = s[3] * e + src[3] * g;
  } else {
    // U + iV relaxes as exp(-(a1 - i a3) tau) toward the stationary state
    const double x = -a1 * dtau, y = a3 * dtau;
    const double ex = exp(x), cy = cos(y), sy = sin(y), sh = sin(0.5 * y);
    const Cx<double> ez{ex * cy, ex * sy};
    const Cx<double> em1{expm1(x) * cy - 2.0 * sh * sh, ex * sy};
    const double den = x * x + y * y;
    const Cx<double> phic{(em1.re * x + em1.im * y) / den, (em1.im * x - em1.re * y) / den};
    const Cx<double> Z{s[2], s[3]}, SZ{src[2], src[3]};
    const Cx<double> Zn = cadd(cmul(Z, ez), cscale(cmul(SZ, phic), dtau));
    Un = Zn.re; Vn = Zn.im;
  }
  s[0] = 0.5 * (An + Bn);
  s[1] = 0.5 * (An - Bn);
  s[2] = Un;
  s[3] = Vn;
}

// Stokes vector scattered toward a camera (basis e1 = theta_hat, e2 = phi_hat
// of its direction) by a dipole whose incident coherency is C9 (real xx yy
// zz xy xz yz, imaginary yz zx xy): rho'_ij = h_i^T C conj(h_j) with h_i =
// alpha e_i and the lab polarizability alpha = a_perp 1 + (a_par - a_perp)
// b b^T (b the grain axis), times pf.
template <bool SPHERE>
__device__ __forceinline__ void source_toward(const double C9[9], const Quat<double>& q, const DustDev& D,
                                              const V3<double>& e1, const V3<double>& e2, double pf,
                                              double S[4]) {
  const double Cr[3][3] = {{C9[0], C9[3], C9[4]}, {C9[3], C9[1], C9[5]}, {C9[4], C9[5], C9[2]}};
  const double i6 = C9[6], i7 = C9[7], i8 = C9[8];
  const double Ci[3][3] = {{0.0, i8, -i7}, {-i8, 0.0, i6}, {i7, -i6, 0.0}};
  Cx<double> h1[3], h2[3];
  const double ev1[3] = {e1.x, e1.y, e1.z}, ev2[3] = {e2.x, e2.y, e2.z};
  if (SPHERE) {
#pragma unroll
    for (int k = 0; k < 3; ++k) { h1[k] = {ev1[k], 0.0}; h2[k] = {ev2[k], 0.0}; }
  } else {
    const V3<double> b = from_grain(q, V3<double>{0.0, 0.0, 1.0});
    const double bv[3] = {b.x, b.y, b.z};
    const double b1 = dot(b, e1), b2 = dot(b, e2);
    const Cx<double> ap{D.ap_re, D.ap_im}, dd{D.aa_re - D.ap_re, D.aa_im - D.ap_im};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      h1[k] = cadd(cscale(ap, ev1[k]), cscale(dd, b1 * bv[k]));
      h2[k] = cadd(cscale(ap, ev2[k]), cscale(dd, b2 * bv[k]));
    }
  }
  // g_j = C conj(h_j)
  Cx<double> g1[3], g2[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    g1[k] = {0.0, 0.0};
    g2[k] = {0.0, 0.0};
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const Cx<double> C{Cr[k][l], Ci[k][l]};
      g1[k] = cadd(g1[k], cmulc(C, h1[l]));
      g2[k] = cadd(g2[k], cmulc(C, h2[l]));
    }
  }
  double r11 = 0.0, r22 = 0.0;
  Cx<double> r12{0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r11 += cmul(h1[k], g1[k]).re;
    r22 += cmul(h2[k], g2[k]).re;
    r12 = cadd(r12, cmul(h1[k], g2[k]));
  }
  S[0] = pf * (r11 + r22);
  S[1] = pf * (r11 - r22);
  S[2] = pf * 2.0 * r12.re;
  S[3] = -pf * 2.0 * r12.im;
}

// Peel-off imaging at a scattering event (the Monte Carlo imaging that Sec.
// 2.3 sets two-step imaging against): for every camera, the Stokes vector the
// event scatters toward it per unit solid angle (from the packet's incident
// coherency, as step 2 forms its source from the tallied one), carried to
// the grid's edge through the Appendix A extinction of every cell on the way
// (no source), added to the pixel the event projects to, per unit pixel
// area.  FP64; open boundaries.
template <typename R, bool ALIGNED, bool SPHERE, bool TAB, bool MESH>
__device__ void peel_off(const Packet<R>& p, const TransportArgs& a, const Quat<double>& q_ev,
                         const DustDev& D) {
  double C9[9];
  const double s_in[4] = {(double)p.I, (double)p.Q, (double)p.U, (double)p.V};
  if (!TAB) coherency<double, 9>(V3<double>{p.nx, p.ny, p.nz}, s_in[0], s_in[1], s_in[2], s_in[3], 1.0, C9);
  double X[3] = {a.x0 + ((double)p.ci + p.fx) * a.dx, a.y0 + ((double)p.cj + p.fy) * a.dx,
                 a.z0 + ((double)p.ck + p.fz) * a.dx};
  if (MESH) {
    // the event's position from its leaf's corner, in finest cells
    const int4 o = reinterpret_cast<const int4*>(a.mesh.leaf_org)[p.leaf];
    const double sz = (double)(1ll << (a.mesh.max_level - o.w));
    X[0] = a.x0 + ((double)o.x + ((double)p.ci + p.fx) * sz) * a.mesh.fine;
    X[1] = a.y0 + ((double)o.y + ((double)p.cj + p.fy) * sz) * a.mesh.fine;
    X[2] = a.z0 + ((double)o.z + ((double)p.ck + p.fz) * sz) * a.mesh.fine;
  }
  const int nn[3] = {a.nx, a.ny, a.nz};
  for (int v = 0; v < a.n_views; ++v) {
    const ViewDev vw = a.views[v];
    const double W = vw.half_width;
    const double xi = X[0] * vw.px + X[1] * vw.py + X[2] * vw.pz;
    const double yi = -(X[0] * vw.tx + X[1] * vw.ty + X[2] * vw.tz);
    const double fxp = (xi + W) / (2.0 * W / a.npx), fyp = (yi + W) / (2.0 * W / a.npy);
    if (!(fxp >= 0.0 && fxp < (double)a.npx && fyp >= 0.0 && fyp < (double)a.npy)) continue;
    const int ix = (int)fxp, iy = (int)fyp;
    const V3<double> Om{vw.ox, vw.oy, vw.oz};
    double st[4];
    if (TAB)
      tab_toward(D, V3<double>{p.nx, p.ny, p.nz}, s_in, Om, V3<double>{vw.tx, vw.ty, vw.tz},
                 V3<double>{vw.px, vw.py, vw.pz}, st);
    else
      source_toward<SPHERE>(C9, q_ev, D, V3<double>{vw.tx, vw.ty, vw.tz}, V3<double>{vw.px, vw.py, vw.pz},
                            D.pfac, st);
    const double om[3] = {vw.ox, vw.oy, vw.oz};
    int ci[3] = {p.ci, p.cj, p.ck};
    double f[3] = {p.fx, p.fy, p.fz};
    int leaf = MESH ? p.leaf : 0, lvl = MESH ? p.lvl : 0;
    const uint64_t Bm = MESH ? (uint64_t)a.mesh.block : 0;
    while (true) {
      double tb = __builtin_huge_val();
      int axis = -1;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        double t;
        if (om[k] > 0.0) t = (1.0 - f[k]) / om[k];
        else if (om[k] < 0.0) t = -f[k] / om[k];
        else continue;
        if (t < tb) { tb = t; axis = k; }
      }
      if (axis < 0) break;
      const uint64_t c = MESH ? (uint64_t)leaf * Bm * Bm * Bm + (uint64_t)ci[0] + Bm * ((uint64_t)ci[1] + Bm * ci[2])
                              : (uint64_t)ci[0] + (uint64_t)a.nx * ((uint64_t)ci[1] + (uint64_t)a.ny * ci[2]);
      const double rho = (double)a.rho[c];
      if (rho > 0.0 && tb > 0.0) {
        const double dtau = rho * D.kext * tb * (MESH ? ldexp(a.dx, -lvl) : a.dx);
        if (SPHERE && !ALIGNED) {
          const double E = exp(-dtau);
#pragma unroll
          for (int k = 0; k < 4; ++k) st[k] *= E;
        } else {
          const double* blk =
              a.tally + ((uint64_t)p.lam * a.nslot + tally_slot(c, ci[0], ci[1], ci[2], MESH ? 0 : a.tbx, a.tby)) *
                            TallyShape<SPHERE>::TS;
          Quat<double> qc{1.0, 0.0, 0.0, 0.0};
          if (ALIGNED) qc = cell_quat<ALIGNED, SPHERE>(a, blk, c);
          V3<double> og = Om;
          double c2 = 1.0, s2 = 0.0;
          if (ALIGNED) {
            og = to_grain(qc, Om);
            eta2(qc, Om, og, c2, s2);
          }
          double a1, a2, a3;
          alphas<double, SPHERE>(D, og.z, a1, a2, a3);
          double sg[4] = {st[0], c2 * st[1] + s2 * st[2], -s2 * st[1] + c2 * st[2], st[3]};
          const double zero[4] = {0.0, 0.0, 0.0, 0.0};
          appA_eigen(a1, a2, a3, dtau, zero, sg);
          st[0] = sg[0];
          st[1] = c2 * sg[1] - s2 * sg[2];
          st[2] = s2 * sg[1] + c2 * sg[2];
          st[3] = sg[3];
        }
      }
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (k != axis) f[k] = fmin(1.0, fmax(0.0, f[k] + tb * om[k]));
      if (om[axis] > 0.0) { ci[axis]++; f[axis] = 0.0; } else { ci[axis]--; f[axis] = 1.0; }
      if (MESH) {
        if ((ci[axis] < 0 || ci[axis] >= (int)Bm) && !mesh_ray_cross(a.mesh, leaf, lvl, ci, f, om)) break;
        continue;
      }
      if (ci[axis] < 0 || ci[axis] >= nn[axis]) break;
    }
    const double area = (2.0 * W / a.npx) * (2.0 * W / a.npy);
    double* out = a.peel + (((uint64_t)p.lam * a.n_views + v) * 4) * ((uint64_t)a.npx * a.npy) +
                  (uint64_t)iy * a.npx + ix;
#pragma unroll
    for (int k = 0; k < 4; ++k) unsafeAtomicAdd(out + (uint64_t)k * a.npx * a.npy, st[k] / area);
  }
}

// Per-view flush of tabulated grains (the scattering source S of Sec. 2.3,
// eq. scat-disc-sum, one Stokes vector per camera): each staged entry holds
// the segment's weighted Stokes integral (lab basis of its direction) and the
// direction.  The wavefront takes the (entry, camera) pairs 64 at a time, one
// per lane, and projects the entry on the camera with the table; the four
// components then go through the wavefront's LDS area `sp` (64 x 4 doubles)
// so that each atomic instruction writes 64 consecutive doubles: the pairs of
// one entry are adjacent in S[lambda][cell][view][4], so an instruction
// covers whole 128-byte lines (two per entry with 8 cameras) instead of
// putting one component of every pair on its own line -- the drain is bound
// by the L2's atomic line requests, and this cuts them four-fold.  Reached by
// all lanes of the wavefront.  The source is per unit volume of the entry's
// cell: on a composite mesh a cell of level l has (dx 2^-l)^3.
template <bool MESH>
__device__ void wave_drain_views(const TransportArgs& a, double* sv, long long* sk, double* sp, int lane,
                                 int& staged) {
  constexpr int NV = 7;  // staged values per entry: weighted J (4) and n (3)
  const int n = staged;
  if (n == 0) return;
  staged = 0;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int nv = a.n_views;
  const int items = n * nv;
  const double inv_vol = 1.0 / (a.dx * a.dx * a.dx);
  for (int base = 0; base < items; base += 64) {
    const int it = base + lane;
    double st[4] = {0.0, 0.0, 0.0, 0.0};
    double iv = inv_vol;
    if (it < items) {
      const int e = it / nv, v = it - e * nv;
      const double* x = sv + e * NV;
      const uint64_t key = (uint64_t)sk[e];
      const DustDev& D = a.dust[key / a.nslot];
      const ViewDev& vw = a.views[v];
      const double s_in[4] = {x[0], x[1], x[2], x[3]};
      tab_toward(D, V3<double>{x[4], x[5], x[6]}, s_in, V3<double>{vw.ox, vw.oy, vw.oz},
                 V3<double>{vw.tx, vw.ty, vw.tz}, V3<double>{vw.px, vw.py, vw.pz}, st);
      if (MESH) {
        const uint64_t b = (uint64_t)a.mesh.block;
        iv = ldexp(inv_vol, 3 * a.mesh.leaf_org[4 * ((key % a.nslot) / (b * b * b)) + 3]);
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) sp[4 * lane + k] = st[k] * iv;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int d = 64 * j + lane;      // component d & 3 of pair d >> 2 of this round
      const int pit = base + (d >> 2);
      const double val = sp[d];
      if (pit < items && val != 0.0) {
        const int e = pit / nv, v = pit - e * nv;
        unsafeAtomicAdd(a.tally + ((uint64_t)sk[e] * nv + v) * 4 + (d & 3), val);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// Scattering event at the packet's current position (Sec. 2.2), the next
// scattering depth, and the roulette check that follows every segment.
template <typename R, bool ALIGNED, bool SPHERE, bool PEEL, bool TAB, bool MESH>
__device__ uint32_t scatter_step(Packet<R>& p, const TransportArgs& a) {
  const uint64_t c = cell_index<MESH>(p, a);
  const DustDev& D = a.dust[p.lam];
  Quat<R> q{(R)1, (R)0, (R)0, (R)0};
  Quat<double> qd{1.0, 0.0, 0.0, 0.0};
  if (ALIGNED) {
    const double* blk =
        a.tally + ((uint64_t)p.lam * a.nslot + tally_slot(c, p.ci, p.cj, p.ck, MESH ? 0 : a.tbx, a.tby)) *
                      TallyShape<SPHERE>::TS;
    qd = cell_quat<ALIGNED, SPHERE>(a, blk, c);
    q = quat_cast<R>(qd);
  }
  if (PEEL) peel_off<R, ALIGNED, SPHERE, TAB, MESH>(p, a, qd, D);
  if (TAB) {
    if (!scatter_tab<R>(p, D, a.seed)) return END_NUMERIC;
  } else if (!scatter<R, ALIGNED, SPHERE>(p, q, qd, D, a.seed)) {
    return END_NUMERIC;
  }
  p.events++;
  p.hash = hash_event(p.hash, EV_SCATTER, c);
  p.tau = -log((double)next_uniform(p, a.seed));
  return roulette<MESH>(p, a);
}

// Russian roulette after a segment or an event in the packet's cell (reading
// R8); the cell index is formed only when the check draws
template <bool MESH, typename R>
__device__ uint32_t roulette(Packet<R>& p, const TransportArgs& a) {
  if (!isfinite(p.I)) return END_NUMERIC;
  if (a.rr_wmin > 0.0 && p.I < (R)a.rr_wmin * p.w0) {
    const uint64_t cn = cell_index<MESH>(p, a);
    R u = next_uniform(p, a.seed);
    if (u < (R)a.rr_psurv) {
      const R before = p.I, inv = (R)1 / (R)a.rr_psurv;
      p.I *= inv; p.Q *= inv; p.U *= inv; p.V *= inv;
      p.e_gain += (double)(p.I - before);
      p.rr++;
      p.hash = hash_event(p.hash, EV_RR_SURVIVE, cn);
    } else {
      p.hash = hash_event(p.hash, END_RR_KILL, cn);
      return END_RR_KILL;
    }
  }
  return 0;
}

// stats slots in LDS
enum { SC_STEPS, SC_SCAT, SC_TRIALS, SC_KILL, SC_SURV, SC_ESC, SC_BUDGET, SC_NUM, SC_PACK, SC_FLUSH, SC_N };
enum { SE_EMIT, SE_ESC, SE_ABS, SE_KILL, SE_GAIN, SE_BUDGET, SE_SCAT, SE_N };

template <typename R>
__device__ void finish(const Packet<R>& p, uint32_t end, const TransportArgs& a,
                       unsigned long long* sc, double* se) {
  atomicAdd(&sc[SC_STEPS], (unsigned long long)p.steps);
  atomicAdd(&sc[SC_SCAT], (unsigned long long)p.events);
  atomicAdd(&sc[SC_TRIALS], (unsigned long long)p.trials);
  atomicAdd(&sc[SC_PACK], 1ull);
  if (p.rr) atomicAdd(&sc[SC_SURV], (unsigned long long)p.rr);
  if (end != END_NUMERIC) {
    atomicAdd(&se[SE_ABS], p.e_abs);
    atomicAdd(&se[SE_SCAT], p.e_scat);
    if (p.e_gain != 0.0) atomicAdd(&se[SE_GAIN], p.e_gain);
  }
  switch (end) {
    case END_ESCAPE: atomicAdd(&sc[SC_ESC], 1ull); atomicAdd(&se[SE_ESC], (double)p.I); break;
    case END_RR_KILL: atomicAdd(&sc[SC_KILL], 1ull); atomicAdd(&se[SE_KILL], (double)p.I); break;
    case END_BUDGET: atomicAdd(&sc[SC_BUDGET], 1ull); atomicAdd(&se[SE_BUDGET], (double)p.I); break;
    default: atomicAdd(&sc[SC_NUM], 1ull); break;
  }
  if (a.trace_count && (p.pid % a.trace_stride) == 0 && p.pid / a.trace_stride < a.trace_count) {
    TraceDev& t = a.traces[(uint64_t)p.lam * a.trace_count + p.pid / a.trace_stride];
    t.packet = p.pid;
    t.end_kind = (int32_t)end;
    t.events = p.events;
    t.steps = p.steps;
    t.last_cell = p.last;
    t.n[0] = (double)p.nx; t.n[1] = (double)p.ny; t.n[2] = (double)p.nz;
    t.stokes[0] = (double)p.I; t.stokes[1] = (double)p.Q;
    t.stokes[2] = (double)p.U; t.stokes[3] = (double)p.V;
    t.hash = p.hash;
    t.tau_path = (double)p.tau_path;
  }
}

template <typename R, bool ALIGNED, bool SPHERE, bool PEEL, bool TAB, bool MESH>
__device__ __forceinline__ void transport_body(const TransportArgs& a) {
  constexpr int NC = TallyShape<SPHERE>::NC, TS = TallyShape<SPHERE>::TS;
  __shared__ unsigned long long sc[SC_N];
  __shared__ double se[SE_N];
  // flush staging, one area of FLUSH_CAP entries per wavefront (43 KB per
  // block for spheres, 61 KB for aligned grains: two blocks per CU; 32 KB
  // for tabulated grains, whose entries are the segment's Stokes integral and
  // direction, 7 values).  A wavefront drains its area once it holds more
  // than FLUSH_CAP - 64 entries (a stage adds at most 64), so a drain covers
  // FLUSH_CAP - 63 .. FLUSH_CAP entries.  With the tally in bricks a cap of
  // 192 beat 256 on the 256^3 disk: 726.8 vs 737.9 ms (a cap of 128:
  // 729.2 ms).
  constexpr int NSV = TAB ? 7 : NC;
  constexpr int FLUSH_CAP = TAB ? 128 : 192;
  __shared__ double s_val[4 * FLUSH_CAP * NSV];
  // tabulated grains: per wavefront the projections of one drain round
  __shared__ double s_proj[TAB ? 4 * 256 : 1];
  __shared__ long long s_key[4 * FLUSH_CAP];
  if (threadIdx.x < SC_N) sc[threadIdx.x] = 0ull;
  if (threadIdx.x < SE_N) se[threadIdx.x] = 0.0;
  __syncthreads();

  const int lane = (int)__lane_id();
  const int wv = (int)(threadIdx.x >> 6);
  double* sv = s_val + wv * FLUSH_CAP * NSV;
  double* sp = s_proj + (TAB ? wv * 256 : 0);
  long long* sk = s_key + wv * FLUSH_CAP;
  int staged = 0;  // entries in this wavefront's staging area (uniform)
  Packet<R> p;
  bool active = false, exhausted = false, pending = false;
  int waited = 0;
  int64_t acc_key = -1;
  unsigned long long flushes = 0;  // tally cells flushed by this wavefront
  double acc[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) acc[k] = 0.0;

  // Packet ids reserved by this wavefront, [wnext, wend) (uniform).  With
  // spherical grains a step is short and every wavefront refills its idle
  // lanes often: taking ids one refill at a time from the one counter all
  // wavefronts share serialised them on that counter (disk 256^3, 1e8
  // packets: 1371 ms), taking WAVE_CHUNK at a time does not (860 ms).  The
  // aligned-grain kernels contend less and measured slower with the reserve
  // (batched workload 718 -> 744 ms in FP64, 449 -> 494 ms in FP32), so they
  // take exactly the ids they need.
  constexpr bool CHUNKED = SPHERE;
  constexpr unsigned long long WAVE_CHUNK = 64;
  // a refill hands up to 64 idle lanes ids from one new chunk
  static_assert(WAVE_CHUNK >= 64, "a chunk must cover a whole wavefront");
  unsigned long long wnext = 0, wend = 0;
  bool global_done = false;  // the global counter has passed the total
  while (true) {
    // refill idle lanes; a chunked wavefront keeps refilling while it holds no
    // packet and still reserves ids (all it was handed may have left the grid)
    do {
    if (!exhausted) {
      const unsigned long long idle = __ballot(!active);
      if (idle) {
        const unsigned long long nidle = (unsigned long long)__popcll(idle);
        const int leader = __ffsll((unsigned long long)idle) - 1;
        if (CHUNKED) {
          const unsigned long long rem = wend - wnext;
          const bool refill = rem < nidle && !global_done;
          unsigned long long base = 0;
          if (refill) {
            if (lane == leader) base = atomicAdd(a.counter, WAVE_CHUNK);
            // the leader's value, as a wave-uniform (scalar) value
            const unsigned lo = __builtin_amdgcn_readlane((unsigned)base, leader);
            const unsigned hi = __builtin_amdgcn_readlane((unsigned)(base >> 32), leader);
            base = ((unsigned long long)hi << 32) | lo;
            if (base + WAVE_CHUNK >= a.total) global_done = true;
          }
          if (!active) {
            const unsigned long long r = (unsigned long long)__popcll(idle & ((1ull << lane) - 1ull));
            const bool have = r < rem || refill;
            const unsigned long long g = r < rem ? wnext + r : base + (r - rem);
            if (have && g < a.total) {
              const bool in = init_packet<R, ALIGNED, SPHERE, MESH>(p, g, a);
              atomicAdd(&se[SE_EMIT], (double)p.I);  // the emitted intensity
              if (in) active = true;
              else finish(p, END_ESCAPE, a, sc, se);
            }
          }
          if (refill) {
            wnext = base + (nidle - rem);
            wend = base + WAVE_CHUNK;
          } else {
            wnext += nidle < rem ? nidle : rem;
          }
          if (global_done && (wnext >= wend || wnext >= a.total)) exhausted = true;
        } else {
          unsigned long long base = 0;
          if (lane == leader) base = atomicAdd(a.counter, nidle);
          base = __shfl(base, leader);
          if (!active) {
            const unsigned long long below = idle & ((1ull << lane) - 1ull);
            const unsigned long long g = base + (unsigned long long)__popcll(below);
            if (g < a.total) {
              const bool in = init_packet<R, ALIGNED, SPHERE, MESH>(p, g, a);
              atomicAdd(&se[SE_EMIT], (double)p.I);  // the emitted intensity
              if (in) active = true;
              else finish(p, END_ESCAPE, a, sc, se);
            }
          }
          if (base + nidle >= a.total) exhausted = true;
        }
      }
    }
    } while (CHUNKED && !exhausted && !__any(active));
    if (!__any(active)) break;
    bool has = false;
    int64_t key = -1;
    R cc[NC];
    if (active && !pending) {
      const uint32_t end = step<R, ALIGNED, SPHERE, TAB, MESH>(p, a, has, key, cc, pending);
      if (end) {
        finish(p, end, a, sc, se);
        active = false;
      }
    }
    if (TAB) {
      // tabulated grains: every segment is staged with its direction (a
      // segment's projection on the cameras depends on it)
      const double e7[7] = {(double)cc[0], (double)cc[1], (double)cc[2], (double)cc[3], p.nx, p.ny, p.nz};
      flushes += wave_stage<7>(has, key, e7, sv, sk, lane, staged);
      if (staged > FLUSH_CAP - 64) wave_drain_views<MESH>(a, sv, sk, sp, lane, staged);
    } else {
    // a lane entering another (wavelength, cell) hands its running sum over
    flushes += wave_stage<NC>(has && key != acc_key && acc_key >= 0, acc_key, acc, sv, sk, lane, staged);
    if (staged > FLUSH_CAP - 64) wave_drain<NC, TS>(a.tally, sv, sk, lane, staged);
    if (has) {
      if (key == acc_key) {
#pragma unroll
        for (int k = 0; k < NC; ++k) acc[k] += (double)cc[k];
      } else {
        acc_key = key;
#pragma unroll
        for (int k = 0; k < NC; ++k) acc[k] = (double)cc[k];
      }
    }
    }
    // Scattering events are run for the parked lanes together once enough
    // of them wait (or one has waited long enough, or nothing else can
    // move): the rejection loop then runs for many lanes at once instead of
    // stalling the wavefront for one lane at a time.
    const unsigned long long pm = __ballot(pending);
    if (pm) {
      ++waited;
      const unsigned long long movable = __ballot(active && !pending);
      if (__popcll(pm) >= a.scatter_batch || waited >= a.scatter_wait || movable == 0ull) {
        waited = 0;
        if (pending) {
          pending = false;
          const uint32_t end = scatter_step<R, ALIGNED, SPHERE, PEEL, TAB, MESH>(p, a);
          if (end) {
            finish(p, end, a, sc, se);
            active = false;
          }
        }
      }
    }
  }
  if (TAB) {
    wave_drain_views<MESH>(a, sv, sk, sp, lane, staged);
  } else {
    flushes += wave_stage<NC>(acc_key >= 0, acc_key, acc, sv, sk, lane, staged);
    wave_drain<NC, TS>(a.tally, sv, sk, lane, staged);
  }
  if (lane == 0) atomicAdd(&sc[SC_FLUSH], flushes);
  __syncthreads();
  if (threadIdx.x < SC_N) atomicAdd(&(&a.stats->cell_steps)[threadIdx.x], sc[threadIdx.x]);
  if (threadIdx.x < SE_N) unsafeAtomicAdd(&(&a.stats->e_emitted)[threadIdx.x], se[threadIdx.x]);
}

// The persistent transport kernels.  FP32 variants are held to two waves per
// SIMD (at most 256 registers): the non-spherical FP32 bodies need 264-272
// unconstrained and would run one wave per SIMD; the bound costs them about a
// dozen spills and makes them 1.5x faster.  The FP64 variants need 297-361;
// holding them to two waves spills 50-190 registers and halves their speed,
// so they run unbounded at one wave per SIMD.  PEEL adds peel-off imaging at
// every scattering event (a separate instantiation: the kernels without it
// are unchanged).
template <bool ALIGNED, bool SPHERE, bool PEEL, bool TAB, bool MESH>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_transport32(TransportArgs a) {
  transport_body<float, ALIGNED, SPHERE, PEEL, TAB, MESH>(a);
}
template <bool ALIGNED, bool SPHERE, bool PEEL, bool TAB, bool MESH>
__global__ void __launch_bounds__(256) k_transport64(TransportArgs a) {
  transport_body<double, ALIGNED, SPHERE, PEEL, TAB, MESH>(a);
}

// ---------------------------------------------------------------------------
// Step 2 (Sec. 2.3): one lane per (wavelength, view, pixel).  The ray enters
// the grid box from the far side and is marched cell by cell toward the
// camera; each cell applies the Appendix A solution with the cell's
// extinction for the camera direction and the scattering source formed from
// the coherency tally (or a caller-given per-view source).  FP64 throughout.
// ---------------------------------------------------------------------------
template <bool ALIGNED, bool SPHERE, bool USER_S, bool MESH>
__global__ void __launch_bounds__(256) k_image(ImageArgs a) {
  // No fused multiply-adds: a ray that grazes a cell face (a pixel centre on
  // a face, drifting off it by ~1e-16 per cell) then takes the face-side
  // decisions of a plain (unfused) evaluation of the same expressions.
#pragma clang fp contract(off)
  const uint64_t npix = (uint64_t)a.npx * a.npy;
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t total = npix * a.n_views * a.n_lambda;
  if (idx >= total) return;
  const int ix = (int)(idx % a.npx);
  const int iy = (int)((idx / a.npx) % a.npy);
  const int v = (int)((idx / npix) % a.n_views);
  const int lam = (int)(idx / (npix * a.n_views));
  const ViewDev vw = a.views[v];
  const DustDev& D = a.dust[lam];
  const double W = vw.half_width;
  const double xp = -W + (ix + 0.5) * (2.0 * W / a.npx);
  const double yp = -W + (iy + 0.5) * (2.0 * W / a.npy);
  const double P0[3] = {xp * vw.px - yp * vw.tx, xp * vw.py - yp * vw.ty, xp * vw.pz - yp * vw.tz};
  const double om[3] = {vw.ox, vw.oy, vw.oz};
  const double lo[3] = {a.x0, a.y0, a.z0};
  const int nn[3] = {a.nx, a.ny, a.nz};
  double sn = -__builtin_huge_val(), sf = __builtin_huge_val();
  bool miss = false;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if ((a.boundary >> k) & 1) continue;  // the periodic copies fill the axis
    const double hi = lo[k] + nn[k] * a.dx;
    if (om[k] != 0.0) {
      const double s1 = (lo[k] - P0[k]) / om[k], s2 = (hi - P0[k]) / om[k];
      sn = fmax(sn, fmin(s1, s2));
      sf = fmin(sf, fmax(s1, s2));
    } else if (P0[k] < lo[k] || P0[k] >= hi) {
      miss = true;
    }
  }
  double st[4] = {0.0, 0.0, 0.0, 0.0};
  if (!miss && sn < sf) {
    int ci[3];
    double f[3];
    // composite mesh: the leaf block of the ray, its level and origin
    int leaf = 0, lvl = 0, sh = 0;
    int4 org{0, 0, 0, 0};
    const MeshDev& m = a.mesh;
    const uint64_t B = MESH ? (uint64_t)m.block : 0;
    if (MESH) {
      // the entry point in finest cells, clamped into the domain
      double t[3];
      long long X[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        t[k] = (P0[k] + sn * om[k] - lo[k]) / m.fine;
        X[k] = (long long)floor(t[k]);
        X[k] = X[k] < 0 ? 0 : (X[k] > m.nfine[k] - 1 ? m.nfine[k] - 1 : X[k]);
      }
      leaf = mesh_find(m, X);
      org = reinterpret_cast<const int4*>(m.leaf_org)[leaf];
      lvl = org.w;
      sh = m.max_level - lvl;
      const long long X0[3] = {org.x, org.y, org.z};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const long long i = (X[k] - X0[k]) >> sh;
        ci[k] = (int)i;
        f[k] = fmin(1.0, fmax(0.0, (t[k] - (double)X0[k]) / (double)(1ll << sh) - (double)i));
      }
    }
#pragma unroll
    for (int k = 0; k < 3 && !MESH; ++k) {
      const double t = (P0[k] + sn * om[k] - lo[k]) / a.dx;
      const double fl = floor(t);
      if ((a.boundary >> k) & 1) {
        const long long n = nn[k], i = (long long)fl;
        ci[k] = (int)(((i % n) + n) % n);
        f[k] = fmin(1.0, fmax(0.0, t - fl));
        continue;
      }
      int i = (int)fl;
      i = i < 0 ? 0 : (i > nn[k] - 1 ? nn[k] - 1 : i);
      ci[k] = i;
      f[k] = fmin(1.0, fmax(0.0, t - (double)i));
    }
    const V3<double> Om{om[0], om[1], om[2]};
    const V3<double> e1{vw.tx, vw.ty, vw.tz}, e2{vw.px, vw.py, vw.pz};
    const double kext = D.kext;
    double clen = MESH ? ldexp(a.dx, -lvl) : a.dx;
    double inv_vol = 1.0 / (clen * clen * clen);
    while (true) {
      double tb = __builtin_huge_val();
      int axis = -1;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        double t;
        if (om[k] > 0.0) t = (1.0 - f[k]) / om[k];
        else if (om[k] < 0.0) t = -f[k] / om[k];
        else continue;
        if (t < tb) { tb = t; axis = k; }
      }
      if (axis < 0) break;
      const uint64_t c = MESH ? (uint64_t)leaf * B * B * B + (uint64_t)ci[0] + B * ((uint64_t)ci[1] + B * ci[2])
                              : (uint64_t)ci[0] + (uint64_t)a.nx * ((uint64_t)ci[1] + (uint64_t)a.ny * ci[2]);
      const uint64_t sl = tally_slot(c, ci[0], ci[1], ci[2], MESH ? 0 : a.tbx, a.tby);
      const double rho = (double)a.rho[c];
      if (rho > 0.0) {
        const double ke = rho * kext;
        const double dtau = ke * tb * clen;
        double S[4];
        Quat<double> q{1.0, 0.0, 0.0, 0.0};
        if (ALIGNED) q = grain_quat(V3<double>{(double)a.bx[c], (double)a.by[c], (double)a.bz[c]});
        if (USER_S) {
          const double* Sv = a.user_S + (((uint64_t)lam * a.nslot + sl) * a.n_views + v) * 4;
          S[0] = Sv[0]; S[1] = Sv[1]; S[2] = Sv[2]; S[3] = Sv[3];
        } else {
          // source toward the camera from the incident coherency C of the
          // cell: rho'_ij = h_i^T C conj(h_j), h_i = alpha e_i with the lab
          // polarizability alpha = a_perp 1 + (a_par - a_perp) b b^T.
          constexpr int TS = TallyShape<SPHERE>::TS;
          const double* T = a.tally + ((uint64_t)lam * a.nslot + sl) * TS;
          double C9[9] = {T[0], T[1], T[2], T[3], T[4], T[5], 0.0, 0.0, 0.0};
          if (TallyShape<SPHERE>::NC == 9) { C9[6] = T[6]; C9[7] = T[7]; C9[8] = T[8]; }
          source_toward<SPHERE>(C9, q, D, e1, e2, D.pfac * inv_vol, S);
        }
        const double ik = 1.0 / ke;
        double src[4] = {S[0] * ik, S[1] * ik, S[2] * ik, S[3] * ik};
        // the dust's thermal emission per unit optical depth,
        // (kappa_abs / kappa_ext) (alpha1, alpha2, 0, 0) B in the grain-frame
        // basis of the ray (eq. polarized-rt)
        const double eB = a.em_B ? D.ka_cell / D.ke_cell * (double)a.em_B[(uint64_t)lam * a.ncell + c] : 0.0;
        if (SPHERE && !ALIGNED) {
          src[0] += eB;
          const double E = exp(-dtau), G = dtau * phi1(dtau);
#pragma unroll
          for (int k = 0; k < 4; ++k) st[k] = st[k] * E + src[k] * G;
        } else {
          V3<double> og = Om;
          double c2 = 1.0, s2 = 0.0;
          if (ALIGNED) {
            og = to_grain(q, Om);
            eta2(q, Om, og, c2, s2);
          }
          double a1, a2, a3;
          alphas<double, SPHERE>(D, og.z, a1, a2, a3);
          double sg[4] = {st[0], c2 * st[1] + s2 * st[2], -s2 * st[1] + c2 * st[2], st[3]};
          const double srcg[4] = {src[0] + eB * a1, c2 * src[1] + s2 * src[2] + eB * a2,
                                  -s2 * src[1] + c2 * src[2], src[3]};
          appA_eigen(a1, a2, a3, dtau, srcg, sg);
          st[0] = sg[0];
          st[1] = c2 * sg[1] - s2 * sg[2];
          st[2] = s2 * sg[1] + c2 * sg[2];
          st[3] = sg[3];
        }
      }
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (k != axis) f[k] = fmin(1.0, fmax(0.0, f[k] + tb * om[k]));
      if (om[axis] > 0.0) { ci[axis]++; f[axis] = 0.0; } else { ci[axis]--; f[axis] = 1.0; }
      if (MESH) {
        if (ci[axis] >= 0 && ci[axis] < (int)B) continue;
        // the leaf beyond the block face (finest-cell units, face rule)
        const double sz = (double)(1ll << sh);
        const long long X0[3] = {org.x, org.y, org.z};
        double t[3];
        long long X[3];
        bool left = false;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          t[k] = (double)X0[k] + ((double)ci[k] + f[k]) * sz;
          X[k] = finest_cell(t[k], om[k]);
          left = left || X[k] < 0 || X[k] >= m.nfine[k];
        }
        if (left) break;
        leaf = mesh_find(m, X);
        org = reinterpret_cast<const int4*>(m.leaf_org)[leaf];
        lvl = org.w;
        sh = m.max_level - lvl;
        const long long X1[3] = {org.x, org.y, org.z};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const long long i = (X[k] - X1[k]) >> sh;
          ci[k] = (int)i;
          f[k] = fmin(1.0, fmax(0.0, (t[k] - (double)X1[k]) / (double)(1ll << sh) - (double)i));
        }
        clen = ldexp(a.dx, -lvl);
        inv_vol = 1.0 / (clen * clen * clen);
        continue;
      }
      if (ci[axis] < 0 || ci[axis] >= nn[axis]) {
        if (!((a.boundary >> axis) & 1)) break;
        ci[axis] = ci[axis] < 0 ? nn[axis] - 1 : 0;
      }
    }
  }
  double* out = a.images + (((uint64_t)lam * a.n_views + v) * 4) * npix + (uint64_t)iy * a.npx + ix;
#pragma unroll
  for (int k = 0; k < 4; ++k) out[(uint64_t)k * npix] = st[k];
}

// ---------------------------------------------------------------------------
// utility kernels
// ---------------------------------------------------------------------------
__global__ void k_fill_zero(uint64_t* p, uint64_t nwords, unsigned char* tail, int ntail) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += stride)
    p[i] = 0ull;
  if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

// Tally blocks before a transport run: coherency slots zero and, with co_b
// (non-spherical grains), the density in slot nc and the grain-frame
// quaternion of the alignment direction (identity without one) in slots
// nc+1..nc+4, for every (wavelength, cell) at its tally slot; the rest of
// each block, and the padding slots of the bricks (never read), zero.  One
// thread per double of a wavelength's tally (ts = 2^lts doubles per slot),
// written for every wavelength: consecutive lanes write consecutive doubles.
__global__ void k_tally_init(double* tally, const float* rho, const float* bx, const float* by,
                             const float* bz, uint64_t ncell, int n_lambda, int lts, int nc, int co_b,
                             uint64_t nslot, int nx, int ny, int tbx, int tby) {
  const int ts = 1 << lts;
  const uint64_t per = nslot << lts;  // doubles per wavelength
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t cxy = (uint64_t)nx * (uint64_t)ny;
  const uint64_t nz = tbx ? ncell / cxy : 0;
  for (uint64_t o = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; o < per; o += stride) {
    const uint64_t sl = o >> lts;
    const int k = (int)(o & (uint64_t)(ts - 1));
    double v = 0.0;
    if (co_b && k >= nc && k <= nc + 4) {
      // the cell of slot sl (the inverse of tally_slot), if it is one
      uint64_t c = sl;
      bool valid = sl < ncell;
      if (tbx) {
        const uint64_t brick = sl >> 6, t = brick / (uint64_t)tbx;
        const int w = (int)(sl & 63);
        const uint64_t i = (brick - t * (uint64_t)tbx) * 4 + (uint64_t)(w & 3);
        const uint64_t j = (t % (uint64_t)tby) * 4 + (uint64_t)((w >> 2) & 3);
        const uint64_t kz = (t / (uint64_t)tby) * 4 + (uint64_t)(w >> 4);
        valid = i < (uint64_t)nx && j < (uint64_t)ny && kz < nz;
        c = i + (uint64_t)nx * j + cxy * kz;
      }
      if (valid) {
        if (k == nc) {
          v = (double)rho[c];
        } else {
          Quat<double> q{1.0, 0.0, 0.0, 0.0};
          if (bx) q = grain_quat(V3<double>{(double)bx[c], (double)by[c], (double)bz[c]});
          const int m = k - nc - 1;
          v = m == 0 ? q.w : (m == 1 ? q.x : (m == 2 ? q.y : q.z));
        }
      }
    }
    for (int lam = 0; lam < n_lambda; ++lam) tally[(uint64_t)lam * per + o] = v;
  }
}

__global__ void k_validate(const float* rho, const float* bx, const float* by, const float* bz,
                           uint64_t n, unsigned long long* bad) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  unsigned long long nbad = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float r = rho[i];
    if (!(r >= 0.0f) || !isfinite(r)) nbad++;
    if (bx) {
      const double b2 = (double)bx[i] * bx[i] + (double)by[i] * by[i] + (double)bz[i] * bz[i];
      if (!(fabs(sqrt(b2) - 1.0) <= 1e-5)) nbad++;
    }
  }
  if (nbad) atomicAdd(bad, nbad);
}

// ---------------------------------------------------------------------------
// Thermal emission tables (set-up of the dust's emission, Sec. 2.2): for one
// wavelength the running sum F of the cell luminosities fac rho B (fac =
// 4 pi kappa_abs dx^3) over the cells in flat order, and its guide table.
// On a composite mesh (lorg non-null: leaf origins and levels, b3 = block^3
// cells per leaf) a cell's luminosity carries its own volume, 2^-3 level of
// a root cell's.  Blocks of EM_CHUNK cells; thread t of a block sums EM_PER
// consecutive cells.
// ---------------------------------------------------------------------------
constexpr int EM_THREADS = 256;
constexpr int EM_PER = 16;
constexpr uint64_t EM_CHUNK = (uint64_t)EM_THREADS * EM_PER;

__device__ __forceinline__ double em_lum(const float* rho, const float* B, double fac, const int32_t* lorg,
                                         uint64_t b3, uint64_t c) {
  const double l = fac * (double)rho[c] * (double)B[c];
  return lorg ? ldexp(l, -3 * lorg[4 * (c / b3) + 3]) : l;
}

__device__ __forceinline__ double em_thread_sum(const float* rho, const float* B, double fac,
                                                const int32_t* lorg, uint64_t b3, uint64_t first,
                                                uint64_t ncell) {
  double sum = 0.0;
  for (int k = 0; k < EM_PER; ++k) {
    const uint64_t c = first + k;
    if (c < ncell) sum += em_lum(rho, B, fac, lorg, b3, c);
  }
  return sum;
}

// exclusive scan of one value per thread over a block of EM_THREADS
__device__ __forceinline__ double em_block_exclusive(double v, double* sh, double* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < EM_THREADS; off <<= 1) {
    const double add = t >= off ? sh[t - off] : 0.0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  const double incl = sh[t];
  *total = sh[EM_THREADS - 1];
  __syncthreads();
  return incl - v;
}

__global__ void __launch_bounds__(EM_THREADS)
k_em_partial(const float* rho, const float* B, double fac, const int32_t* lorg, uint64_t b3, uint64_t ncell,
             double* partial) {
  __shared__ double sh[EM_THREADS];
  const uint64_t first = (uint64_t)blockIdx.x * EM_CHUNK + (uint64_t)threadIdx.x * EM_PER;
  double total;
  em_block_exclusive(em_thread_sum(rho, B, fac, lorg, b3, first, ncell), sh, &total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// one block: block totals -> exclusive block offsets, in place
__global__ void __launch_bounds__(EM_THREADS) k_em_offsets(double* partial, uint64_t nb) {
  __shared__ double sh[EM_THREADS];
  const uint64_t per = (nb + EM_THREADS - 1) / EM_THREADS;
  const uint64_t b0 = (uint64_t)threadIdx.x * per;
  double sum = 0.0;
  for (uint64_t b = b0; b < b0 + per && b < nb; ++b) sum += partial[b];
  double total;
  double run = em_block_exclusive(sum, sh, &total);
  for (uint64_t b = b0; b < b0 + per && b < nb; ++b) {
    const double v = partial[b];
    partial[b] = run;
    run += v;
  }
}

__global__ void __launch_bounds__(EM_THREADS)
k_em_cdf(const float* rho, const float* B, double fac, const int32_t* lorg, uint64_t b3, uint64_t ncell,
         const double* offsets, double* cdf) {
  __shared__ double sh[EM_THREADS];
  const uint64_t first = (uint64_t)blockIdx.x * EM_CHUNK + (uint64_t)threadIdx.x * EM_PER;
  double total;
  double run = offsets[blockIdx.x] +
               em_block_exclusive(em_thread_sum(rho, B, fac, lorg, b3, first, ncell), sh, &total);
  for (int k = 0; k < EM_PER; ++k) {
    const uint64_t c = first + k;
    if (c < ncell) {
      run += em_lum(rho, B, fac, lorg, b3, c);
      cdf[c] = run;
    }
  }
}

// guide[k] = the first cell whose running sum exceeds L k / ncell
// (k < ncell); guide[ncell] = the last cell
__global__ void k_em_guide(const double* cdf, uint64_t ncell, uint32_t* guide) {
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k > ncell) return;
  if (k == ncell) { guide[k] = (uint32_t)(ncell - 1); return; }
  const double T = cdf[ncell - 1] * ((double)k / (double)ncell);
  uint64_t lo = 0, hi = ncell - 1;
  while (lo < hi) {
    const uint64_t mid = lo + ((hi - lo) >> 1);
    if (T < cdf[mid]) hi = mid; else lo = mid + 1;
  }
  guide[k] = (uint32_t)lo;
}

uint64_t emission_blocks(uint64_t ncell) { return (ncell + EM_CHUNK - 1) / EM_CHUNK; }

hipError_t launch_emission_table(const float* rho, const float* B, double fac, const int32_t* leaf_org,
                                 uint64_t block3, uint64_t ncell, double* partial, double* cdf, uint32_t* guide,
                                 hipStream_t s) {
  const uint64_t nb = emission_blocks(ncell);
  hipLaunchKernelGGL(k_em_partial, dim3((unsigned)nb), dim3(EM_THREADS), 0, s, rho, B, fac, leaf_org, block3,
                     ncell, partial);
  hipLaunchKernelGGL(k_em_offsets, dim3(1), dim3(EM_THREADS), 0, s, partial, nb);
  hipLaunchKernelGGL(k_em_cdf, dim3((unsigned)nb), dim3(EM_THREADS), 0, s, rho, B, fac, leaf_org, block3, ncell,
                     (const double*)partial, cdf);
  hipLaunchKernelGGL(k_em_guide, dim3((unsigned)((ncell + 1 + 255) / 256)), dim3(256), 0, s,
                     (const double*)cdf, ncell, guide);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <bool A, bool S, bool T, bool M>
static void launch_one(const TransportArgs& a, bool fp64, bool peel, int blocks, int bs, hipStream_t s) {
  if (fp64 && peel) hipLaunchKernelGGL((k_transport64<A, S, true, T, M>), dim3(blocks), dim3(bs), 0, s, a);
  else if (fp64) hipLaunchKernelGGL((k_transport64<A, S, false, T, M>), dim3(blocks), dim3(bs), 0, s, a);
  else if (peel) hipLaunchKernelGGL((k_transport32<A, S, true, T, M>), dim3(blocks), dim3(bs), 0, s, a);
  else hipLaunchKernelGGL((k_transport32<A, S, false, T, M>), dim3(blocks), dim3(bs), 0, s, a);
}



hipError_t launch_transport(const TransportArgs& a, bool fp64, bool aligned, bool sphere, bool peel, bool tab,
                            bool mesh, int blocks, int block_size, hipStream_t s) {
  if (mesh && tab) {
    launch_one<false, true, true, true>(a, fp64, peel, blocks, block_size, s);
  } else if (mesh) {
    if (aligned && sphere) launch_one<true, true, false, true>(a, fp64, peel, blocks, block_size, s);
    else if (aligned) launch_one<true, false, false, true>(a, fp64, peel, blocks, block_size, s);
    else if (sphere) launch_one<false, true, false, true>(a, fp64, peel, blocks, block_size, s);
    else launch_one<false, false, false, true>(a, fp64, peel, blocks, block_size, s);
  } else if (tab) {
    launch_one<false, true, true, false>(a, fp64, peel, blocks, block_size, s);
  } else if (aligned && sphere) {
    launch_one<true, true, false, false>(a, fp64, peel, blocks, block_size, s);
  } else if (aligned) {
    launch_one<true, false, false, false>(a, fp64, peel, blocks, block_size, s);
  } else if (sphere) {
    launch_one<false, true, false, false>(a, fp64, peel, blocks, block_size, s);
  } else {
    launch_one<false, false, false, false>(a, fp64, peel, blocks, block_size, s);
  }
  return hipGetLastError();
}

template <bool A, bool S, bool PL, bool T, bool M>
static int occ_one(bool fp64, int bs) {
  int n = 0;
  const hipError_t e = fp64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_transport64<A, S, PL, T, M>, bs, 0)
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_transport32<A, S, PL, T, M>, bs, 0);
  return e == hipSuccess ? n : 0;
}

template <bool A, bool S, bool T, bool M>
static int occ_peel(bool fp64, bool peel, int bs) {
  return peel ? occ_one<A, S, true, T, M>(fp64, bs) : occ_one<A, S, false, T, M>(fp64, bs);
}

int transport_max_blocks_per_cu(bool fp64, bool aligned, bool sphere, bool peel, bool tab, bool mesh,
                                int block_size) {
  if (mesh && tab) return occ_peel<false, true, true, true>(fp64, peel, block_size);
  if (mesh) {
    if (aligned && sphere) return occ_peel<true, true, false, true>(fp64, peel, block_size);
    if (aligned) return occ_peel<true, false, false, true>(fp64, peel, block_size);
    if (sphere) return occ_peel<false, true, false, true>(fp64, peel, block_size);
    return occ_peel<false, false, false, true>(fp64, peel, block_size);
  }
  if (tab) return occ_peel<false, true, true, false>(fp64, peel, block_size);
  if (aligned && sphere) return occ_peel<true, true, false, false>(fp64, peel, block_size);
  if (aligned) return occ_peel<true, false, false, false>(fp64, peel, block_size);
  if (sphere) return occ_peel<false, true, false, false>(fp64, peel, block_size);
  return occ_peel<false, false, false, false>(fp64, peel, block_size);
}

template <bool U, bool M>
static void launch_image_one(const ImageArgs& a, bool aligned, bool sphere, dim3 grid, int bs, hipStream_t s) {
  if (aligned && sphere) hipLaunchKernelGGL((k_image<true, true, U, M>), grid, dim3(bs), 0, s, a);
  else if (aligned) hipLaunchKernelGGL((k_image<true, false, U, M>), grid, dim3(bs), 0, s, a);
  else if (sphere) hipLaunchKernelGGL((k_image<false, true, U, M>), grid, dim3(bs), 0, s, a);
  else hipLaunchKernelGGL((k_image<false, false, U, M>), grid, dim3(bs), 0, s, a);
}

hipError_t launch_image(const ImageArgs& a, bool aligned, bool sphere, bool user_source, bool mesh,
                        hipStream_t s) {
  const uint64_t total = (uint64_t)a.npx * a.npy * a.n_views * a.n_lambda;
  const int bs = 128;
  const dim3 grid((unsigned)((total + bs - 1) / bs));
  if (user_source && mesh) launch_image_one<true, true>(a, aligned, sphere, grid, bs, s);
  else if (user_source) launch_image_one<true, false>(a, aligned, sphere, grid, bs, s);
  else if (mesh) launch_image_one<false, true>(a, aligned, sphere, grid, bs, s);
  else launch_image_one<false, false>(a, aligned, sphere, grid, bs, s);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  const uint64_t nwords = bytes / 8;
  const int ntail = (int)(bytes % 8);
  uint64_t blocks = (nwords + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, (uint64_t*)p, nwords,
                     (unsigned char*)p + nwords * 8, ntail);
  return hipGetLastError();
}

hipError_t launch_tally_init(double* tally, const float* rho, const float* bx, const float* by,
                             const float* bz, uint64_t ncell, int n_lambda, bool sphere, uint64_t nslot, int nx,
                             int ny, int tbx, int tby, hipStream_t s) {
  const int ts = tally_stride(sphere), nc = tally_components(sphere);
  const int co_b = sphere ? 0 : 1;
  int lts = 0;
  while ((1 << lts) < ts) ++lts;
  if ((1 << lts) != ts || (co_b && nc + 5 > ts)) return hipErrorInvalidValue;
  uint64_t blocks = ((nslot << lts) + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_tally_init, dim3((unsigned)blocks), dim3(256), 0, s, tally, rho, bx, by, bz, ncell,
                     n_lambda, lts, nc, co_b, nslot, nx, ny, tbx, tby);
  return hipGetLastError();
}

hipError_t launch_validate(const float* rho, const float* bx, const float* by, const float* bz,
                           uint64_t n, unsigned long long* bad, hipStream_t s) {
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_validate, dim3((unsigned)blocks), dim3(256), 0, s, rho, bx, by, bz, n, bad);
  return hipGetLastError();
}

}  // namespace kp
