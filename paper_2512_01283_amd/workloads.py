"""Seeded synthetic inputs for the transport and imaging path.

This module only builds input arrays and parameter records (density grids,
alignment fields, grain polarizabilities, sources, cameras, packet counts).
It holds none of the transport or imaging arithmetic, and it is the only
module that both the HIP path and the CPU oracle consume.

A workload is a plain dict:
  grid    {nx, ny, nz, x0, y0, z0, dx[, boundary]}  cubic cells, lower corner
          (x0, y0, z0); boundary: bit a set = axis a (x, y, z) periodic
  rho     float32[nz*ny*nx]             density, x fastest
  bhat    float32[3, ncell] or None     unit grain-alignment direction per cell
  dust    list (one per wavelength) of {kappa_sca, kappa_abs, a_perp, a_par,
          alpha3_scale}; kappas per unit density per unit length
  source  {kind (0 isotropic point, 1 pencil, 2 the dust's thermal emission),
          pos, dir, lum}
  emission float32[n_lambda, ncell]     (kind 2 only) source function B of
          every cell at each wavelength
  views   list of {theta, phi, npx, npy, half_width}
  packets list (one per wavelength) of packet counts
  opts    {seed, rr_wmin, rr_psurv, max_events}
  precision "f64" | "f32"  (arithmetic of the Monte Carlo step)
"""
from __future__ import annotations

import math

import numpy as np

DEG = math.pi / 180.0


# --------------------------------------------------------------------------
# grain polarizabilities (input parameters, not part of the transport)
# --------------------------------------------------------------------------
def oblate_depolarization(aspect: float) -> tuple[float, float]:
    """Depolarization factors (L_long, L_short) of an oblate spheroid with
    axis ratio `aspect` = long/short (Bohren & Huffman 1983, Sec. 5.3).
    The two long axes share L_long; L_long*2 + L_short = 1."""
    e2 = 1.0 - 1.0 / aspect ** 2
    g = math.sqrt((1.0 - e2) / e2)
    l_long = g / (2.0 * e2) * (math.pi / 2.0 - math.atan(g)) - g * g / 2.0
    return l_long, 1.0 - 2.0 * l_long


def dipole_polarizabilities(m: complex, aspect: float) -> tuple[complex, complex]:
    """(a_perp, a_par) of a perfectly aligned oblate spheroid in the dipole
    approximation, a_j = (eps-1)/(1+L_j(eps-1)) (common volume factor dropped:
    only ratios enter).  a_perp is across the symmetry (short) axis, which is
    the alignment direction; a_par is along it."""
    eps = m * m
    l_long, l_short = oblate_depolarization(aspect)
    return (eps - 1) / (1 + l_long * (eps - 1)), (eps - 1) / (1 + l_short * (eps - 1))


def sphere_dust(kappa_ext: float, albedo: float) -> dict:
    return dict(kappa_sca=albedo * kappa_ext, kappa_abs=(1.0 - albedo) * kappa_ext,
                a_perp=1.0 + 0j, a_par=1.0 + 0j, alpha3_scale=0.0)


def oblate_dust(kappa_ext: float, albedo: float, m=2.30 + 0.0228j, aspect=2.0,
                alpha3_scale=0.0) -> dict:
    ap, aa = dipole_polarizabilities(m, aspect)
    return dict(kappa_sca=albedo * kappa_ext, kappa_abs=(1.0 - albedo) * kappa_ext,
                a_perp=complex(ap), a_par=complex(aa), alpha3_scale=alpha3_scale)


def table_nodes(n_theta: int) -> np.ndarray:
    """cos Theta at the nodes of a scattering table: Theta uniform on [0, pi]."""
    return np.cos(np.linspace(0.0, math.pi, int(n_theta)))


def hg_table(g=0.5, p_lin=0.5, p_circ=0.2, n_theta=361) -> np.ndarray:
    """An analytic scattering-plane table [n_theta][6] (S11 S12 S22 S33 S34
    S44): a Henyey-Greenstein S11 of asymmetry g with Rayleigh-shaped
    polarisation of peak p_lin, a circular term of peak p_circ (S34), and
    S22 = S11, S44 = S33 (S12^2 + S33^2 + S34^2 <= S11^2 when
    p_lin^2 + p_circ^2 <= 1)."""
    mu = table_nodes(n_theta)
    s11 = (1.0 - g * g) / (1.0 + g * g - 2.0 * g * mu) ** 1.5
    f = (1.0 - mu * mu) / (1.0 + mu * mu)
    c = 2.0 * mu / (1.0 + mu * mu)
    return np.stack([s11, -p_lin * s11 * f, s11, s11 * c, p_circ * s11 * f, s11 * c], axis=1)


def rayleigh_table(n_theta=181) -> np.ndarray:
    """The Rayleigh scattering-plane table (amplitude functions S1 = 1,
    S2 = cos Theta), any scale."""
    mu = table_nodes(n_theta)
    return np.stack([1 + mu * mu, mu * mu - 1, 1 + mu * mu, 2 * mu, 0 * mu, 2 * mu], axis=1)


def table_dust(kappa_ext: float, albedo: float, table: np.ndarray) -> dict:
    """Grains with a tabulated scattering matrix and scalar extinction."""
    return dict(sphere_dust(kappa_ext, albedo), table=np.ascontiguousarray(table, dtype=np.float64))


def default_opts(seed: int) -> dict:
    return dict(seed=int(seed), rr_wmin=1e-3, rr_psurv=0.1, max_events=10000)


def _centres(n: int, x0: float, dx: float) -> np.ndarray:
    return x0 + (np.arange(n) + 0.5) * dx


def _cube(n: int):
    dx = 2.0 / n
    return dict(nx=n, ny=n, nz=n, x0=-1.0, y0=-1.0, z0=-1.0, dx=dx)


def _mesh(grid):
    x = _centres(grid["nx"], grid["x0"], grid["dx"])
    y = _centres(grid["ny"], grid["y0"], grid["dx"])
    z = _centres(grid["nz"], grid["z0"], grid["dx"])
    return np.meshgrid(x, y, z, indexing="ij")  # arrays indexed [i, j, k]


def _flat(a_ijk: np.ndarray) -> np.ndarray:
    """[i, j, k] -> flat x-fastest float32."""
    return np.ascontiguousarray(np.transpose(a_ijk, (2, 1, 0)), dtype=np.float32).reshape(-1)


def view(theta_deg, phi_deg, npix, half_width=1.0):
    return dict(theta=theta_deg * DEG, phi=phi_deg * DEG, npx=npix, npy=npix,
                half_width=half_width)


# --------------------------------------------------------------------------
# the five headline workloads
# --------------------------------------------------------------------------
def uniform_sphere(n=32, packets=100_000, albedo=1.0, tau_radius=1.0, seed=0,
                   views=None, npix=64) -> dict:
    """Uniform sphere of radius 1 on an n^3 grid over [-1,1]^3 (density 1 where
    the cell centre lies inside), radial optical depth `tau_radius`, Rayleigh
    spheres, isotropic unpolarised star at the centre (a grid vertex)."""
    grid = _cube(n)
    X, Y, Z = _mesh(grid)
    rho = (X * X + Y * Y + Z * Z < 1.0).astype(np.float64)
    return dict(name=f"sphere{n}", grid=grid, rho=_flat(rho), bhat=None,
                dust=[sphere_dust(tau_radius, albedo)],
                source=dict(kind=0, pos=(0.0, 0.0, 0.0), dir=(0.0, 0.0, 1.0), lum=1.0),
                views=views if views is not None else [view(90.0, 0.0, npix)],
                packets=[int(packets)], opts=default_opts(seed), precision="f64")


def mesh_tree(rx, ry, rz, block, max_level, refine):
    """The child array of a composite mesh (roots first, x fastest; the 8
    children of a refined node consecutive, octant bit 0 = upper x half,
    bit 1 = y, bit 2 = z; -1 = leaf) and, per node, (level, lower corner in
    finest cells).  refine(level, corner, edge) decides, for a block at
    `level` with lower corner and edge in finest cells, whether it is split
    (never beyond max_level)."""
    full = block << max_level
    child = []
    info = []
    for r in range(rx * ry * rz):
        child.append(-1)
        info.append((0, (r % rx * full, r // rx % ry * full, r // (rx * ry) * full)))
    i = 0
    while i < len(child):
        lev, org = info[i]
        if lev < max_level and refine(lev, org, full >> lev):
            child[i] = len(child)
            half = full >> (lev + 1)
            for k in range(8):
                child.append(-1)
                info.append((lev + 1, (org[0] + (k & 1) * half, org[1] + ((k >> 1) & 1) * half,
                                       org[2] + ((k >> 2) & 1) * half)))
        i += 1
    return np.array(child, dtype=np.int32), info


def mesh_cells(grid) -> tuple[np.ndarray, np.ndarray]:
    """Centres [ncell, 3] and levels [ncell] of the cells of grid["mesh"] in
    flat order (leaves in node order, cells x fastest within a leaf)."""
    m = grid["mesh"]
    B, L = int(m["block"]), int(m["max_level"])
    child = np.asarray(m["child"])
    full = B << L
    rx, ry, rz = int(m["rx"]), int(m["ry"]), int(m["rz"])
    info = [(0, (r % rx * full, r // rx % ry * full, r // (rx * ry) * full)) for r in range(rx * ry * rz)]
    info += [None] * (len(child) - len(info))
    for i, c in enumerate(child):  # children follow their parents
        if c >= 0:
            lev, org = info[i]
            half = full >> (lev + 1)
            for k in range(8):
                info[c + k] = (lev + 1, (org[0] + (k & 1) * half, org[1] + ((k >> 1) & 1) * half,
                                         org[2] + ((k >> 2) & 1) * half))
    fine = grid["dx"] / (1 << L)
    k = np.arange(B)
    loc = np.stack(np.meshgrid(k, k, k, indexing="ij"), axis=-1)[..., ::-1].reshape(-1, 3)  # x fastest
    cen, lev = [], []
    for node in np.nonzero(child == -1)[0]:
        l, org = info[node]
        sz = 1 << (L - l)
        cen.append(np.array([grid["x0"], grid["y0"], grid["z0"]]) + (np.array(org) + (loc + 0.5) * sz) * fine)
        lev.append(np.full(B ** 3, l))
    return np.concatenate(cen), np.concatenate(lev)


def make_mesh_grid(x0, y0, z0, dx, rx, ry, rz, block, max_level, refine) -> dict:
    """A grid record with a composite mesh: root cells of size dx, rx*ry*rz
    root blocks of block^3 cells, refined by refine (see mesh_tree)."""
    child, _ = mesh_tree(rx, ry, rz, block, max_level, refine)
    return dict(nx=rx * block, ny=ry * block, nz=rz * block, x0=x0, y0=y0, z0=z0, dx=dx,
                mesh=dict(rx=rx, ry=ry, rz=rz, block=block, max_level=max_level, child=child))


def mesh_sphere(rx=4, block=8, max_level=2, packets=100_000, albedo=1.0, tau_radius=1.0, seed=12,
                views=None, npix=32) -> dict:
    """The uniform sphere of radius 1 in [-1,1]^3 (density 1 where a cell's
    centre lies inside) on a composite mesh refined toward the central star:
    blocks reaching within 0.6 of the centre split to level 1, within 0.3 to
    level 2."""
    n = rx * block
    reach = (0.6, 0.3, 0.15)

    def refine(lev, org, edge):
        fine = 2.0 / (n << max_level)
        lo = -1.0 + np.array(org) * fine
        hi = lo + edge * fine
        d = np.linalg.norm(np.maximum(0.0, np.maximum(lo, -hi)))  # distance from the centre to the block
        return d < reach[min(lev, 2)]

    grid = make_mesh_grid(-1.0, -1.0, -1.0, 2.0 / n, rx, rx, rx, block, max_level, refine)
    cen, _ = mesh_cells(grid)
    rho = (np.einsum("ij,ij->i", cen, cen) < 1.0).astype(np.float32) * np.float32(tau_radius)
    return dict(name=f"mesh_sphere{n}", grid=grid, rho=rho, bhat=None,
                dust=[sphere_dust(1.0, albedo)],
                source=dict(kind=0, pos=(0.0, 0.0, 0.0), dir=(0.0, 0.0, 1.0), lum=1.0),
                views=views if views is not None else [view(90.0, 0.0, npix), view(30.0, 40.0, npix)],
                packets=[int(packets)], opts=default_opts(seed), precision="f64")


def mesh_of_uniform(cfg, block, max_level, p_split=0.4, seed=0) -> dict:
    """The same medium as the uniform grid of cfg (nx divisible by block)
    on a composite mesh refined at random (each block split with probability
    p_split): every cell takes the density (and alignment and thermal source
    function) of the root cell holding it, so the optical properties are the
    same function of position."""
    g = cfg["grid"]
    rx, ry, rz = g["nx"] // block, g["ny"] // block, g["nz"] // block
    rng = np.random.default_rng(seed)
    grid = make_mesh_grid(g["x0"], g["y0"], g["z0"], g["dx"], rx, ry, rz, block, max_level,
                          lambda lev, org, edge: rng.uniform() < p_split)
    cen, _ = mesh_cells(grid)
    ijk = np.floor((cen - np.array([g["x0"], g["y0"], g["z0"]])) / g["dx"]).astype(np.int64)
    root = ijk[:, 0] + g["nx"] * (ijk[:, 1] + g["ny"] * ijk[:, 2])
    out = dict(cfg, grid=grid, rho=np.ascontiguousarray(np.asarray(cfg["rho"])[root], dtype=np.float32))
    if cfg.get("bhat") is not None:
        out["bhat"] = np.ascontiguousarray(np.asarray(cfg["bhat"])[:, root], dtype=np.float32)
    if cfg.get("emission") is not None:
        out["emission"] = np.ascontiguousarray(np.asarray(cfg["emission"])[:, root], dtype=np.float32)
    out["name"] = cfg["name"] + "_mesh"
    return out


def table_sphere(n=32, packets=100_000, albedo=1.0, tau_radius=1.0, g=0.5, seed=11,
                 views=None, npix=32, n_theta=361) -> dict:
    """The uniform sphere of uniform_sphere with grains of tabulated
    scattering (hg_table of asymmetry g)."""
    cfg = uniform_sphere(n=n, packets=packets, albedo=albedo, tau_radius=tau_radius, seed=seed,
                         views=views, npix=npix)
    cfg["name"] = f"table_sphere{n}"
    cfg["dust"] = [table_dust(tau_radius, albedo, hg_table(g, n_theta=n_theta))]
    return cfg


def slab_clump(n=128, packets=10_000_000, seed=1, npix=None) -> dict:
    """Slab |z| <= 0.25 of log-normal density (sigma_ln = 1; a Gaussian random
    field from white noise smoothed over 2 cells and re-standardised; median
    cell optical depth 0.02) plus a Gaussian clump at (0.4, 0, 0) of radius
    0.05 with peak cell optical depth 100; cell optical depths clipped to
    [1e-3, 100] inside the slab.  Oblate 2:1 grains (m = 2.30 + 0.0228i)
    aligned with a uniform field tilted 45 deg from z toward x; albedo 0.5."""
    from scipy.ndimage import gaussian_filter

    grid = _cube(n)
    dx = grid["dx"]
    X, Y, Z = _mesh(grid)
    rng = np.random.Generator(np.random.Philox(seed))
    g = gaussian_filter(rng.standard_normal((n, n, n)), sigma=2.0, mode="wrap")
    g = (g - g.mean()) / g.std()
    kext = 1.0
    tau_med = 0.02
    tau_grf = tau_med * np.exp(g)                  # median tau_med, sigma_ln 1
    r2c = (X - 0.4) ** 2 + Y ** 2 + Z ** 2
    tau_clump = 100.0 * np.exp(-r2c / (2 * 0.05 ** 2))
    tau = np.clip(tau_grf + tau_clump, 1e-3, 100.0)
    rho = np.where(np.abs(Z) <= 0.25, tau / (kext * dx), 0.0)
    b = np.array([math.sin(45 * DEG), 0.0, math.cos(45 * DEG)])
    ncell = n ** 3
    bhat = np.repeat(b[:, None], ncell, axis=1).astype(np.float32)
    npix = npix or n
    return dict(name=f"slab_clump{n}", grid=grid, rho=_flat(rho), bhat=bhat,
                dust=[oblate_dust(kext, 0.5)],
                source=dict(kind=0, pos=(0.0, 0.0, 0.0), dir=(0.0, 0.0, 1.0), lum=1.0),
                views=[view(t, 0.0, npix) for t in (0.0, 30.0, 60.0, 90.0)],
                packets=[int(packets)], opts=default_opts(seed), precision="f32")


def disk_density(grid, h0=0.1, r_in=0.05, r_out=1.0, tau_mid=1.0e4):
    """Flared disk rho ~ r^-1 exp(-z^2/2h^2), h/r = h0 (r/r_out)^0.25,
    zero outside r_in <= r <= r_out (cylindrical r at cell centres).
    Returns (rho, kappa_ext) with kappa_ext set so that the midplane optical
    depth summed over the cells just above the +x axis is tau_mid."""
    X, Y, Z = _mesh(grid)
    r = np.sqrt(X * X + Y * Y)
    h = h0 * r * (r / r_out) ** 0.25
    with np.errstate(divide="ignore", invalid="ignore"):
        rho = np.where((r >= r_in) & (r <= r_out), np.exp(-Z * Z / (2 * h * h)) / r, 0.0)
    rho32 = rho.astype(np.float32)
    j0, k0 = grid["ny"] // 2, grid["nz"] // 2
    column = rho32[grid["nx"] // 2:, j0, k0].astype(np.float64).sum() * grid["dx"]
    return rho32, tau_mid / column


def flared_disk(n=256, packets=100_000_000, seed=2, n_views=8, npix=None, albedo=0.5,
                h0=0.1, tau_mid=1.0e4) -> dict:
    """Flared protoplanetary disk on n^3 over [-1,1]^3, Rayleigh spheres,
    central star, two-step imaging at n_views inclinations from 0 to 90 deg."""
    grid = _cube(n)
    rho, kext = disk_density(grid, h0=h0, tau_mid=tau_mid)
    npix = npix or n
    views = [view(k * 90.0 / max(n_views - 1, 1), 0.0, npix) for k in range(n_views)]
    return dict(name=f"disk{n}", grid=grid, rho=_flat(rho), bhat=None,
                dust=[sphere_dust(kext, albedo)],
                source=dict(kind=0, pos=(0.0, 0.0, 0.0), dir=(0.0, 0.0, 1.0), lum=1.0),
                views=views, packets=[int(packets)], opts=default_opts(seed),
                precision="f32")


def table_disk(n=256, packets=100_000_000, seed=2, n_views=8, npix=None, g=0.5) -> dict:
    """The flared disk of flared_disk with grains of tabulated scattering
    (hg_table of asymmetry g, 181 nodes): every segment is projected on
    every camera (the per-view source)."""
    cfg = flared_disk(n=n, packets=packets, seed=seed, n_views=n_views, npix=npix)
    d = cfg["dust"][0]
    cfg["dust"] = [table_dust(d["kappa_sca"] + d["kappa_abs"], d["kappa_sca"] / (d["kappa_sca"] + d["kappa_abs"]),
                              hg_table(g, n_theta=181))]
    cfg["name"] = f"table_disk{n}"
    return cfg


def bitrev5(k: int) -> int:
    return int(f"{k:05b}"[::-1], 2)


def batched_lambda_counts(n_lambda=32, n_min=1.0e6, ratio=30.0):
    return [int(round(n_min * ratio ** (bitrev5(k) / 31.0))) for k in range(n_lambda)]


def helical_field(grid, pitch_deg=30.0) -> np.ndarray:
    """B = cos(pitch) phi_hat_cyl + sin(pitch) z_hat at cell centres."""
    X, Y, Z = _mesh(grid)
    r = np.sqrt(X * X + Y * Y)
    c, s = math.cos(pitch_deg * DEG), math.sin(pitch_deg * DEG)
    bx, by, bz = -c * Y / r, c * X / r, np.full_like(r, s)
    return np.stack([_flat(bx), _flat(by), _flat(bz)]).astype(np.float32)


def batched_disk(n=256, n_lambda=32, seed=3, npix=None, counts=None) -> dict:
    """Disk density with a helical field (pitch 30 deg) and aligned oblate
    grains at n_lambda wavelengths, lambda_k = lambda_0 10^(k/31), opacities
    kappa(lambda) = kappa(lambda_0) (lambda/lambda_0)^-1.5, uneven packet
    counts 1e6 * 30^(bitrev5(k)/31); 16 views."""
    grid = _cube(n)
    rho, kext0 = disk_density(grid)
    npix = npix or n
    dust = [oblate_dust(kext0 * 10.0 ** (-1.5 * k / 31.0), 0.5) for k in range(n_lambda)]
    views = [view(t, p, npix) for t in (15.0, 40.0, 65.0, 90.0) for p in (0.0, 90.0, 180.0, 270.0)]
    return dict(name=f"batched_disk{n}x{n_lambda}", grid=grid, rho=_flat(rho),
                bhat=helical_field(grid), dust=dust,
                source=dict(kind=0, pos=(0.0, 0.0, 0.0), dir=(0.0, 0.0, 1.0), lum=1.0),
                views=views,
                packets=counts if counts is not None else batched_lambda_counts(n_lambda),
                opts=default_opts(seed), precision="f32")


# --------------------------------------------------------------------------
# small verification workloads (pins and parity cases)
# --------------------------------------------------------------------------
def pencil_slab(n_z=256, tau_total=1.0, p0=0.01, alpha3_scale=0.0, twist=True,
                start_tau=1.0, nxy=2) -> dict:
    """Plane slab of optical depth tau_total along z with dichroic grains whose
    alignment lies in the xy plane; twist=True rotates it as
    (cos 2 pi tau, sin 2 pi tau, 0) with depth tau (Sec. 3.2), else it is
    fixed along x.  A pencil beam starts at depth start_tau and travels -z.
    Grains are given a_perp, a_par with Im ratio chosen so that the
    polarization efficiency across the axis is p0."""
    dz = tau_total / n_z
    grid = dict(nx=nxy, ny=nxy, nz=n_z, x0=-nxy * dz / 2, y0=-nxy * dz / 2, z0=0.0, dx=dz)
    zc = (np.arange(n_z) + 0.5) * dz
    ang = 2 * math.pi * zc if twist else np.zeros(n_z)
    b = np.stack([np.cos(ang), np.sin(ang), np.zeros(n_z)])
    bhat = np.repeat(b[:, :, None], nxy * nxy, axis=2).reshape(3, -1).astype(np.float32)
    rho = np.ones(nxy * nxy * n_z, dtype=np.float32)
    # across the axis: alpha2/alpha1 = (Im a_par - Im a_perp)/(Im a_par + Im a_perp) = -p0
    im_perp, im_par = 1.0 + p0, 1.0 - p0
    dust = dict(kappa_sca=0.0, kappa_abs=1.0, a_perp=complex(1.0, im_perp),
                a_par=complex(1.0, im_par), alpha3_scale=alpha3_scale)
    # kappa_ext per unit length so that alpha1 (across the axis) = 1 in units of tau
    c_avg = (2 * im_perp + im_par) / 3.0
    a1 = (im_par + im_perp) / (2 * c_avg)
    dust["kappa_abs"] = 1.0 / a1
    return dict(name="pencil_slab", grid=grid, rho=rho, bhat=bhat, dust=[dust],
                source=dict(kind=1, pos=(0.0, 0.0, start_tau), dir=(0.0, 0.0, -1.0), lum=1.0),
                views=[view(0.0, 0.0, 4)], packets=[1],
                opts=dict(default_opts(0), rr_wmin=0.0), precision="f64")


# --------------------------------------------------------------------------
# thermal emission of the dust (source kind 2)
# --------------------------------------------------------------------------
THERMAL_SOURCE = dict(kind=2, pos=(0.0, 0.0, 0.0), dir=(0.0, 0.0, 1.0), lum=1.0)


def _isothermal(rho, n_lambda=1, B=1.0):
    """Source function B of every cell, the same everywhere (isothermal
    dust; B in units of the Planck function at the dust temperature)."""
    return np.full((n_lambda, rho.size), B, dtype=np.float32)


def thermal_cube(n=32, packets=1_000_000, tau_half=20.0, albedo=0.5, seed=5, npix=32) -> dict:
    """Isothermal cube of uniform density filling [-1,1]^3, optical depth
    tau_half from the centre to a face, Rayleigh spheres, the dust's thermal
    emission as the only source, one face-on view."""
    grid = _cube(n)
    rho = np.ones(n ** 3, dtype=np.float32)
    return dict(name=f"thermal_cube{n}", grid=grid, rho=rho, bhat=None,
                dust=[sphere_dust(tau_half, albedo)], source=dict(THERMAL_SOURCE),
                emission=_isothermal(rho), views=[view(0.0, 0.0, npix)],
                packets=[int(packets)], opts=default_opts(seed), precision="f64")


def thermal_sphere(n=64, packets=100_000, tau_radius=1.0, albedo=0.0, seed=6, npix=32) -> dict:
    """Isothermal uniform sphere of radius 1 (density 1 where the cell centre
    lies inside), radial optical depth tau_radius, Rayleigh spheres, thermal
    emission as the only source (pure absorption by default)."""
    grid = _cube(n)
    X, Y, Z = _mesh(grid)
    rho = _flat((X * X + Y * Y + Z * Z < 1.0).astype(np.float64))
    return dict(name=f"thermal_sphere{n}", grid=grid, rho=rho, bhat=None,
                dust=[sphere_dust(tau_radius, albedo)], source=dict(THERMAL_SOURCE),
                emission=_isothermal(rho), views=[view(90.0, 0.0, npix)],
                packets=[int(packets)], opts=default_opts(seed), precision="f64")


def emission_slab(tau_total=1.0, p0=0.3, n_z=16, nxy=4, packets=2000, albedo=0.0) -> dict:
    """Uniformly aligned, isothermal dichroic slab (Sec. 3.3): the grains of
    pencil_slab (alignment along x, polarization efficiency p0 across it),
    optical depth tau_total along z, thermal emission as the only source,
    viewed along z.  With albedo 0 its image is eq. ptau in every pixel."""
    cfg = pencil_slab(n_z=n_z, tau_total=tau_total, p0=p0, twist=False, start_tau=tau_total, nxy=nxy)
    d = dict(cfg["dust"][0])
    kext = d["kappa_abs"]
    d["kappa_sca"], d["kappa_abs"] = albedo * kext, (1.0 - albedo) * kext
    g = cfg["grid"]
    cfg.update(name="emission_slab", dust=[d], source=dict(THERMAL_SOURCE),
               emission=_isothermal(cfg["rho"]), packets=[int(packets)],
               views=[dict(theta=0.0, phi=0.0, npx=nxy, npy=nxy, half_width=nxy * g["dx"] / 2)],
               opts=dict(default_opts(7), rr_wmin=0.0))
    return cfg


def dust_cylinder(n=128, packets=10_000_000, tau_axis=1.0, r0=0.25, albedo=0.5, aligned=False,
                  seed=8, npix=None) -> dict:
    """The isothermal dust cylinder of Sec. 3.1 (self-scattering of thermal
    emission): axis along x, rho = rho0 exp(-(r/r0)^2) with r the distance
    from the axis, optical depth tau_axis through the axis along z
    (rho0 kappa r0 sqrt(pi)); Rayleigh spheres, or with aligned=True oblate
    grains aligned along y (across the axis, in the sky plane of the face-on
    view); thermal emission as the only source.  Views: face-on (along z)
    and 60 deg from it toward x."""
    grid = _cube(n)
    X, Y, Z = _mesh(grid)
    rho = _flat(np.exp(-(Y * Y + Z * Z) / r0 ** 2))
    kext = tau_axis / (r0 * math.sqrt(math.pi))
    npix = npix or n
    bhat = None
    dust = sphere_dust(kext, albedo)
    if aligned:
        bhat = np.zeros((3, rho.size), dtype=np.float32)
        bhat[1] = 1.0
        dust = oblate_dust(kext, albedo)
    return dict(name=f"dust_cylinder{n}", grid=grid, rho=rho, bhat=bhat, dust=[dust],
                source=dict(THERMAL_SOURCE), emission=_isothermal(rho),
                views=[view(0.0, 0.0, npix), view(60.0, 0.0, npix)],
                packets=[int(packets)], opts=default_opts(seed), precision="f32")


def periodic_slab(n=16, n_z=16, tau=1.0, albedo=0.0, packets=100_000, views=((0.0, 0.0), (60.0, 30.0)),
                  npix=8, seed=9) -> dict:
    """Isothermal slab of uniform density and optical thickness tau along z,
    periodic in x and y (an infinite slab), Rayleigh spheres, thermal
    emission as the only source; face-on and inclined views."""
    dz = 1.0 / n_z
    grid = dict(nx=n, ny=n, nz=n_z, x0=-n * dz / 2, y0=-n * dz / 2, z0=0.0, dx=dz, boundary=3)
    rho = np.ones(n * n * n_z, dtype=np.float32)
    return dict(name="periodic_slab", grid=grid, rho=rho, bhat=None,
                dust=[sphere_dust(tau, albedo)], source=dict(THERMAL_SOURCE),
                emission=_isothermal(rho), views=[view(t, p, npix, half_width=0.75) for t, p in views],
                packets=[int(packets)], opts=default_opts(seed), precision="f64")


def pencil_column(n_z=64, tau=0.02, packets=1_000_000, npix=16, seed=10) -> dict:
    """A column one cell wide and n_z cells tall of optical depth tau
    (Rayleigh spheres, albedo 1) with a pencil beam entering at the bottom
    along +z, seen edge-on from +x: single scattering at exactly 90 degrees
    toward the camera."""
    dz = 1.0 / n_z
    grid = dict(nx=1, ny=1, nz=n_z, x0=-dz / 2, y0=-dz / 2, z0=-0.5, dx=dz)
    rho = np.ones(n_z, dtype=np.float32)
    return dict(name="pencil_column", grid=grid, rho=rho, bhat=None, dust=[sphere_dust(tau, 1.0)],
                source=dict(kind=1, pos=(0.0, 0.0, -0.5), dir=(0.0, 0.0, 1.0), lum=1.0),
                views=[dict(theta=90.0 * DEG, phi=0.0, npx=1, npy=npix, half_width=0.5)],
                packets=[int(packets)], opts=dict(default_opts(seed), rr_wmin=0.0), precision="f64")


# --------------------------------------------------------------------------
# denoiser inputs: parameter initialisation, synthetic maps, training disks
# --------------------------------------------------------------------------
DN_WIDTHS = (48, 96, 192)


def denoiser_layer_io(widths=DN_WIDTHS, cin=4):
    """(input, output) channels of each 3x3 convolution, in parameter order:
    encoder blocks, the bottleneck, decoder blocks (two convolutions each)."""
    c = list(widths)
    L = len(c)
    io = []
    for l in range(L - 1):
        io += [(cin if l == 0 else c[l - 1], c[l]), (c[l], c[l])]
    io += [(c[L - 2], c[L - 1]), (c[L - 1], c[L - 1])]
    for l in range(L - 2, -1, -1):
        io += [(c[l + 1] + c[l], c[l]), (c[l], c[l])]
    return io


def denoiser_params(seed=0, widths=DN_WIDTHS, bias_std=0.0, head_std=0.0, cin=4) -> np.ndarray:
    """Flat FP32 parameter vector: He-normal 3x3 weights [cout][3][3][cin]
    (std sqrt(2 / (9 cin))) and N(0, bias_std) biases for each convolution,
    then the head [2][c1] ~ N(0, head_std) and its bias N(0, bias_std).  With
    head_std = 0 the untrained network is the identity on Q and U.  cin is
    the number of input features (8 for two-run inputs)."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, cout in denoiser_layer_io(widths, cin):
        parts.append(rng.standard_normal(cout * 9 * ci) * math.sqrt(2.0 / (9 * ci)))
        parts.append(rng.standard_normal(cout) * bias_std)
    parts.append(rng.standard_normal(2 * widths[0]) * head_std)
    parts.append(rng.standard_normal(2) * bias_std)
    return np.concatenate(parts).astype(np.float32)


def synthetic_stokes_maps(seed, batch, height, width, p_max=0.3, noise=0.1, runs=1) -> np.ndarray:
    """[batch, 4, height, width] FP64 Stokes maps with the structure of a
    scattered-light image: I a smooth positive blob plus a floor, a
    polarization fraction up to p_max with a smoothly varying angle, V small,
    and multiplicative noise of relative size `noise`; I is raised where the
    noise would leave I < |(Q, U, V)|.  With runs = 2: [batch, 8, height,
    width], two realisations of each scene with independent noise (the
    first run's four maps, then the second's)."""
    rng = np.random.default_rng(seed)
    yy, xx = np.meshgrid(np.linspace(-1, 1, height), np.linspace(-1, 1, width), indexing="ij")
    out = np.empty((batch, 4 * runs, height, width))
    for b in range(batch):
        cx, cy, r0 = rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3), rng.uniform(0.3, 0.8)
        rr = np.hypot(xx - cx, yy - cy)
        I = np.exp(-(rr / r0) ** 2) + 0.05
        p = p_max * np.clip(rr / r0, 0.0, 1.0)
        chi = np.arctan2(yy - cy, xx - cx) + rng.uniform(0, np.pi)
        for r in range(runs):
            o = out[b, 4 * r:4 * r + 4]
            n = 1.0 + noise * rng.standard_normal((4, height, width))
            o[0] = I * np.abs(n[0])
            o[1] = I * p * np.cos(2 * chi) * n[1]
            o[2] = I * p * np.sin(2 * chi) * n[2]
            o[3] = 0.01 * I * rng.standard_normal((height, width))
            # keep every pixel a physical Stokes vector, I >= |(Q, U, V)|
            o[0] = np.maximum(o[0], 1.001 * np.sqrt((o[1:] ** 2).sum(0)))
    return out


def denoiser_disk(seed, packets, n=256, npix=None) -> dict:
    """One member of the denoiser's training family: the flared disk with
    cos(inclination) ~ U[0, 1] for each of 8 views (azimuth 0), h/r
    prefactor ~ U[0.05, 0.15], and with probability 1/2 aligned oblate grains
    in the helical field, else Rayleigh spheres.  One run images all views."""
    rng = np.random.default_rng([seed, 4])
    h0 = float(rng.uniform(0.05, 0.15))
    aligned = bool(rng.uniform() < 0.5)
    incl = np.degrees(np.arccos(rng.uniform(0.0, 1.0, 8)))
    grid = _cube(n)
    rho, kext = disk_density(grid, h0=h0)
    npix = npix or n
    dust = oblate_dust(kext, 0.5) if aligned else sphere_dust(kext, 0.5)
    return dict(name=f"dn_disk{n}", grid=grid, rho=_flat(rho),
                bhat=helical_field(grid) if aligned else None, dust=[dust],
                source=dict(kind=0, pos=(0.0, 0.0, 0.0), dir=(0.0, 0.0, 1.0), lum=1.0),
                views=[view(float(t), 0.0, npix) for t in incl], packets=[int(packets)],
                opts=default_opts(seed), precision="f32", h0=h0, aligned=aligned)
