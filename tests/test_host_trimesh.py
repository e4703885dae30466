"""The library's host build of triangle-mesh levels (lts_mesh_host) against
the oracle's triangle-mesh levels: DOF, P and F+ flags and lumped masses bit
for bit, fine tiles within the region cap, rejected inputs."""
import numpy as np
import pytest

import meshgen
import paper_2106_11117_amd as P
from oracle import trimesh

MESHES = {"criss_cross": lambda: meshgen.criss_cross(), "delaunay": lambda: meshgen.delaunay_disk(),
          "criss_cross_s1": lambda: meshgen.criss_cross(n=12, ref=2, jitter=0.25, seed=1)}


def _level(m):
    return trimesh.tri_level(m["xy"], m["tris"], m["dirichlet"], m["tri_block"], m["tri_fine"], m["qoi_nodes"],
                             m["n_blocks"], m["h"], m["p"], m["nu"])


@pytest.mark.parametrize("name", list(MESHES))
def test_host_build_matches_oracle(name):
    """The library's host build (lts_mesh_host): DOF, P and F+ flags and lumped
    masses bit for bit as the oracle's; sizes."""
    m = MESHES[name]()
    tl = _level(m)
    trimesh.operators(tl)
    h = P.mesh_host(m)
    fl = h["flags"]
    assert np.array_equal((fl & 1) != 0, ~m["dirichlet"])
    assert np.array_equal((fl & 2) != 0, tl.Pmask)
    assert np.array_equal((fl & 4) != 0, tl.Fplus)
    assert np.array_equal(h["mass"], tl.mass)
    assert (h["n_dof"], h["n_P"], h["n_Fplus"]) == (tl.n_dof, int(tl.Pmask.sum()), int(tl.Fplus.sum()))
    assert h["n_tiles"] >= 1 and h["max_region"] <= P._lib.LTS_MESH_REGION_CAP


def test_host_build_tiles_a_large_F_plus():
    """F+ too large for one region: several tiles, each region within the cap,
    covering F+ (regions at least as large as F+ in total)."""
    m = meshgen.criss_cross(n=48, ref=4, box=(0.3, 0.7))
    h = P.mesh_host(m)
    assert h["n_tiles"] > 1 and h["max_region"] <= P._lib.LTS_MESH_REGION_CAP and h["halo_ratio"] >= 1.0


def test_host_build_rejects_bad_meshes():
    m = meshgen.criss_cross(n=6, ref=2)
    bad = dict(m)
    bad["tris"] = m["tris"][:, [0, 2, 1]]                    # clockwise
    with pytest.raises(P.LtsError):
        P.mesh_host(bad)
    bad = dict(m)
    bad["tri_block"] = m["tri_block"] + 100                  # block out of range
    with pytest.raises(P.LtsError):
        P.mesh_host(bad)
    bad = dict(m)
    bad["p"] = 0
    with pytest.raises(P.LtsError):
        P.mesh_host(bad)
    # a fan of 14 triangles around a fine centre node: degree 14 > 12
    ang = np.linspace(0, 2 * np.pi, 15)[:-1]
    xy = np.concatenate([[[0.0, 0.0]], np.stack([np.cos(ang), np.sin(ang)], 1)])
    tris = np.array([[0, 1 + k, 1 + (k + 1) % 14] for k in range(14)])
    fan = {"xy": xy, "tris": tris, "dirichlet": np.r_[False, np.ones(14, bool)], "tri_block": np.zeros(14, int),
           "tri_fine": np.ones(14, bool), "qoi_nodes": np.zeros(15), "n_blocks": 1, "h": 1.0, "p": 2, "nu": 0.0}
    with pytest.raises(P.LtsError):
        P.mesh_host(fan)
    fan["tri_fine"] = np.zeros(14, bool)                     # not in F+: any degree is fine
    assert P.mesh_host(fan)["n_Fplus"] == 0
