"""Pins of the oracle's composite mesh with static refinement (Sec. 2: the
mesh the packets cross, optionally statically refined; reading M1):

 * a mesh of one unrefined root block is the uniform grid: every packet's
   history (event hash, steps, final state) and the images are identical;
 * a randomly refined mesh carrying the same medium as a uniform grid
   (each cell takes the density of the root cell holding it) gives every
   packet the same history up to rounding (events, end, direction, Stokes
   vector, optical depth travelled: the paths are the same lines through the
   same medium, only cut into more cells), the same volume integral of the
   scattering source per camera, and the same images for a given source
   (Appendix A composes exactly across cells of equal properties);
 * camera rays through refined blocks with a source piecewise constant at
   root resolution give the uniform grid's image to rounding;
 * malformed trees are refused.
"""
import numpy as np
import pytest

from paper_2512_01283_amd import workloads as W


@pytest.fixture(scope="module")
def O():
    from oracle import oracle as o
    o.lib()
    return o


def single_block(cfg):
    g = cfg["grid"]
    n = g["nx"]
    grid = dict(g, mesh=dict(rx=1, ry=1, rz=1, block=n, max_level=0, child=np.array([-1], np.int32)))
    return dict(cfg, grid=grid)


def test_unrefined_single_block_is_the_uniform_grid(O):
    cfg = W.uniform_sphere(n=16, packets=20_000, npix=16, views=[W.view(90, 0, 16), W.view(35, 70, 16)])
    img_u, S_u, tr_u, st_u = O.run(cfg, traces=True)
    img_m, S_m, tr_m, st_m = O.run(single_block(cfg), traces=True)
    for k in ("hash", "end_kind", "events", "steps", "last_cell"):
        assert np.array_equal(tr_u[k], tr_m[k]), k
    assert np.array_equal(tr_u["stokes"], tr_m["stokes"]) and np.array_equal(tr_u["n"], tr_m["n"])
    assert np.array_equal(S_u, S_m) or np.abs(S_u - S_m).max() <= 1e-15 * np.abs(S_u).max()
    assert np.abs(img_u - img_m).max() <= 1e-14 * np.abs(img_u).max()


@pytest.mark.parametrize("block,max_level,aligned", [(4, 2, False), (2, 3, False), (4, 1, True)])
def test_refined_mesh_of_the_same_medium(O, block, max_level, aligned):
    """Same packets through the same medium on the uniform grid and on a
    randomly refined mesh: histories agree to 1e-9 (the mesh cuts each
    segment into more cells, so rounding differs); the source's volume
    integral per camera (sum over cells of S V) agrees to 1e-9.  Roulette is
    off: its check follows every cell segment, so on a finer mesh it would
    draw at other points of the path (reading R8)."""
    if aligned:
        base = W.slab_clump(n=16, packets=4000, npix=16)
        base["views"] = [W.view(90, 0, 16), W.view(35, 70, 16)]
        base["precision"] = "f64"
    else:
        base = W.uniform_sphere(n=16, packets=20_000, npix=16, albedo=0.7,
                                views=[W.view(90, 0, 16), W.view(35, 70, 16)])
    base["opts"] = dict(base["opts"], rr_wmin=0.0)
    mesh = W.mesh_of_uniform(base, block, max_level, p_split=0.45, seed=block + max_level)
    _, S_u, tr_u, st_u = O.run(base, traces=True)
    _, S_m, tr_m, st_m = O.run(mesh, traces=True)
    assert st_m["cell_steps"] > st_u["cell_steps"]  # the refinement is crossed
    for k in ("end_kind", "events"):
        assert np.array_equal(tr_u[k], tr_m[k]), k
    scale = tr_u["stokes"][:, :1]
    assert np.abs(tr_u["stokes"] - tr_m["stokes"]).max(initial=0) <= 1e-9 * max(1.0, scale.max())
    assert (np.abs(tr_u["stokes"] - tr_m["stokes"]) <= 1e-9 * np.abs(scale) + 1e-300).all()
    assert np.abs(tr_u["n"] - tr_m["n"]).max() <= 1e-9
    assert np.allclose(tr_u["tau_path"], tr_m["tau_path"], rtol=1e-9, atol=1e-12)
    # volume integral of the source per camera and component
    g = base["grid"]
    _, lev = W.mesh_cells(mesh["grid"])
    V_m = (g["dx"] / 2.0 ** lev) ** 3
    tot_u = S_u.sum(0) * g["dx"] ** 3
    tot_m = np.einsum("c,cvk->vk", V_m, S_m)
    assert np.abs(tot_u - tot_m).max() <= 1e-9 * np.abs(tot_u[:, 0]).max()


def test_step2_through_refined_blocks(O):
    """A source per unit volume piecewise constant at root resolution
    (S = rho s_v for camera v) imaged through the uniform grid and through a
    randomly refined mesh of the same medium: equal to 1e-12.  The cameras
    are oblique or exactly along an axis: a ray that grazes a face (a pixel
    centre on a face, drifting off it by 1e-16 per cell, as at theta = 90
    degrees where cos theta = 6e-17) may be placed on either side of it by
    the rounding of the mesh's finest-cell coordinates."""
    base = W.uniform_sphere(n=16, packets=1, npix=24, tau_radius=2.0,
                            views=[W.view(123, 211, 24), W.view(35, 70, 24), W.view(0, 0, 24)])
    mesh = W.mesh_of_uniform(base, 4, 2, p_split=0.5, seed=3)
    rng = np.random.default_rng(4)
    s_v = rng.normal(size=(3, 4))
    s_v[:, 0] = np.abs(s_v[:, 0]) + 2.0
    S_u = np.asarray(base["rho"], float)[:, None, None] * s_v[None]
    S_m = np.asarray(mesh["rho"], float)[:, None, None] * s_v[None]
    img_u = O.image(base, S_u)
    img_m = O.image(mesh, S_m)
    d = np.abs(img_u - img_m).max() / np.abs(img_u[:, 0]).max()
    print(f"max |uniform - mesh| / I_max = {d:.2e}")
    assert d < 1e-12
    assert np.abs(img_u[:, 0]).max() > 0


def test_malformed_meshes_are_refused(O):
    cfg = W.mesh_of_uniform(W.uniform_sphere(n=8, packets=10, npix=8), 4, 1, p_split=1.0, seed=1)
    child = cfg["grid"]["mesh"]["child"]
    bad = []
    c = child.copy(); c[0] = 0; bad.append(c)                # a node its own child
    c = child.copy(); c[1] = c[0]; bad.append(c)             # two parents of the same children
    c = child.copy(); c[0] = len(c) - 4; bad.append(c)       # children beyond the node list
    for ch in bad:
        m = dict(cfg["grid"]["mesh"], child=ch)
        with pytest.raises(ValueError):
            O.transport(dict(cfg, grid=dict(cfg["grid"], mesh=m)), tally=False)
    deep = dict(cfg["grid"]["mesh"], max_level=0)            # deeper than max_level
    with pytest.raises(ValueError):
        O.transport(dict(cfg, grid=dict(cfg["grid"], mesh=deep)), tally=False)
    wrong = dict(cfg["grid"], nx=cfg["grid"]["nx"] + 1)      # box not rx * block
    with pytest.raises(ValueError):
        O.transport(dict(cfg, grid=wrong), tally=False)


def test_thermal_emission_on_a_refined_mesh(O):
    """The dust's thermal emission on a randomly refined mesh of the same
    medium and source function: the total luminosity (cell volumes of their
    levels) equals the uniform grid's to 1e-10; the image of the direct
    emission equals the uniform grid's to 1e-12; the escaping fraction of an
    isothermal, purely absorbing sphere is the closed form's within 4 sigma
    (+1e-3), as on the uniform grid; emission cells follow the luminosity."""
    import math
    from test_oracle_emission import escape_probability
    base = W.thermal_sphere(n=32, packets=60_000, tau_radius=1.0, npix=24)
    base["views"] = [W.view(123, 211, 24, half_width=base["views"][0]["half_width"]),
                     W.view(35, 70, 24, half_width=base["views"][0]["half_width"])]
    mesh = W.mesh_of_uniform(base, 4, 2, p_split=0.5, seed=21)
    Lu, Lm = O.emission_luminosity(base), O.emission_luminosity(mesh)
    assert abs(Lm / Lu - 1) < 1e-10, (Lu, Lm)  # running sums over 3e4 and 2e5 cells
    iu, im = O.image(base, None), O.image(mesh, None)
    assert np.abs(iu - im).max() <= 1e-12 * np.abs(iu[:, 0]).max()
    _, _, st = O.transport(mesh, tally=False)
    p = st["e_escaped"] / st["e_emitted"]
    pc = escape_probability(1.0)
    N = mesh["packets"][0]
    sig = math.sqrt(pc * (1 - pc) / N)
    print(f"mesh: escaped fraction {p:.5f}, closed form {pc:.5f} (sigma {sig:.1e}); "
          f"uniform-grid medium 32^3 on a mesh")
    assert abs(p - pc) < 4 * sig + 3e-3  # 32^3 cell-centre sphere: optical radius to ~0.2 %
    # emission cells: histogram of the leaf levels of 4000 emitted packets
    # against each level's share of the luminosity
    _, lev = W.mesh_cells(mesh["grid"])
    B = np.asarray(mesh["emission"])[0]
    dx = mesh["grid"]["dx"]
    lum = np.asarray(mesh["rho"], float) * B * (dx / 2.0 ** lev) ** 3
    cells = np.array([O.emit_state(mesh, k)[0] for k in range(4000)])
    for l in range(3):
        share = lum[lev == l].sum() / lum.sum()
        got = np.mean(lev[cells] == l)
        assert abs(got - share) < 4 * math.sqrt(share * (1 - share) / 4000) + 1e-3, (l, got, share)


@pytest.mark.parametrize("aligned", [False, True])
def test_peel_off_on_a_refined_mesh_of_the_same_medium(O, aligned):
    """Peel-off imaging (reading P1) on a randomly refined mesh of the same
    medium as a uniform grid, roulette off: the same events, seen along the
    same lines through the same medium cut into more cells, give the uniform
    grid's peel-off images to 1e-9 of their maximum.  A single unrefined
    block gives them to 1e-14 (the oracle's threads add their events into
    the images in any order, so even two runs on one grid differ at 1e-16)."""
    if aligned:
        base = W.slab_clump(n=16, packets=3000, npix=16)
        base["precision"] = "f64"
    else:
        base = W.uniform_sphere(n=16, packets=10_000, npix=16, albedo=0.7)
    base["views"] = [W.view(123, 211, 16, half_width=base["views"][0]["half_width"]),
                     W.view(35, 70, 16, half_width=base["views"][0]["half_width"])]
    base["opts"] = dict(base["opts"], rr_wmin=0.0)
    mesh = W.mesh_of_uniform(base, 4, 2, p_split=0.45, seed=31)
    pu, _, st_u = O.transport_peel(base)
    pm, _, st_m = O.transport_peel(mesh)
    assert st_m["cell_steps"] > st_u["cell_steps"] and st_m["scatterings"] == st_u["scatterings"]
    d = np.abs(pu - pm).max() / np.abs(pu[:, 0]).max()
    print(f"peel-off on the mesh: max |uniform - mesh| / I_max = {d:.2e}")
    assert d < 1e-9 and np.abs(pu[:, 0]).max() > 0
    p1, _, _ = O.transport_peel(single_block(base))
    assert np.abs(p1 - pu).max() <= 1e-14 * np.abs(pu[:, 0]).max()


def test_tabulated_grains_on_a_refined_mesh_of_the_same_medium(O):
    """Tabulated scattering (readings T1, T2) on a randomly refined mesh of
    the uniform sphere's medium, roulette off: the same histories to 1e-9,
    and the per-view source's volume integral per camera (sum over cells of
    S V, each cell's volume of its level) equal to 1e-9."""
    base = W.table_sphere(n=16, packets=10_000, tau_radius=1.0, albedo=0.8, g=0.6,
                          views=[W.view(123, 211, 16), W.view(35, 70, 16)])
    base["opts"] = dict(base["opts"], rr_wmin=0.0)
    mesh = W.mesh_of_uniform(base, 4, 2, p_split=0.45, seed=5)
    _, S_u, tr_u, _ = O.run(base, traces=True)
    _, S_m, tr_m, _ = O.run(mesh, traces=True)
    for k in ("end_kind", "events"):
        assert np.array_equal(tr_u[k], tr_m[k]), k
    assert (np.abs(tr_u["stokes"] - tr_m["stokes"]) <= 1e-9 * np.abs(tr_u["stokes"][:, :1]) + 1e-300).all()
    _, lev = W.mesh_cells(mesh["grid"])
    dx = base["grid"]["dx"]
    tot_u = S_u.sum(0) * dx ** 3
    tot_m = np.einsum("c,cvk->vk", (dx / 2.0 ** lev) ** 3, S_m)
    d = np.abs(tot_u - tot_m).max() / np.abs(tot_u[:, 0]).max()
    print(f"tables on the mesh: volume integral of S, max rel. difference {d:.2e}")
    assert d <= 1e-9 and (lev > 0).any()
