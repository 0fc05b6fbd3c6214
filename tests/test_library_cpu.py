"""Host-side checks of libfr.so that need no GPU.

* the library loads and exports every function include/fr.h declares;
* connectivity (neighbour tables) equals the oracle's bit for bit: the two
  use different algorithms (integer corner orientation in the oracle,
  flux-point positions in the library) for the same unique answer;
* invalid meshes are rejected with the documented status codes;
* the device footprint formula matches a direct count.
"""
import os
import re

import numpy as np
import pytest

from oracle.oracle import OracleMesh
from paper_2501_05709_amd import _lib
from paper_2501_05709_amd import workloads as W
from paper_2501_05709_amd.solver import connectivity, footprint

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fr_[a-z_]+)\s*\(", src)) - {"fr_alloc_fn", "fr_free_fn"})


def test_library_exports_every_declared_symbol():
    L = _lib.load()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
        assert n in _lib.SIGNATURES, n


def _rotated_ogrid():
    from tests.test_oracle_pins import ROTATIONS, _face_nodes, _rotate_element
    m = W.naca_ogrid(0.02, 0.4, 0.12, 12, 3, 2)
    m.update(W.airfoil_flow())
    rng = np.random.default_rng(5)
    E = len(m["elem_nodes"])
    perm_e = rng.permutation(E)
    conn = m["elem_nodes"][perm_e].copy()
    for e in range(E):
        conn[e] = _rotate_element(conn[e], 2, ROTATIONS[e % len(ROTATIONS)])
    old_to_new = np.argsort(perm_e)
    bf = []
    for e_old, f, kind in m["bfaces"]:
        e_new = old_to_new[e_old]
        old_nodes = set(m["elem_nodes"][e_old][_face_nodes(f, 2)])
        for f2 in range(6):
            if set(conn[e_new][_face_nodes(f2, 2)]) == old_nodes:
                bf.append((e_new, f2, kind))
    m["elem_nodes"] = conn
    m["bfaces"] = np.array(bf, dtype=np.int64)
    return m


MESHES = {
    "box2d": lambda: W.box_mesh(2, (5, 3), (0, 0), (1.0, 0.7), order=3),
    "box2d_curved": lambda: W.box_mesh(2, (4, 4), (0, 0), (1, 1), q=2, warp=0.05, order=2),
    "box3d": lambda: W.box_mesh(3, (3, 2, 4), (0, 0, 0), (1, 1, 2), order=3),
    "box3d_self_periodic": lambda: W.box_mesh(3, (1, 2, 1), (0, 0, 0), (1, 1, 1), order=2),
    "single_element_2d": lambda: W.box_mesh(2, (1, 1), (0, 0), (1.0, 1.3), order=3),
    "single_element_3d": lambda: W.box_mesh(3, (1, 1, 1), (0, 0, 0), (1.0, 1.3, 0.8), order=3),
    "ragged_box3d_curved": lambda: W.box_mesh(3, (5, 3, 7), (0, 0, 0), (1.0, 0.6, 1.4), q=2, warp=0.04, order=3),
    "ogrid": lambda: dict(W.naca_ogrid(0.04, 0.4, 0.12, 16, 4, 2), **W.airfoil_flow()),
    "ogrid_p4": lambda: dict(W.naca_ogrid(0.0, 0.4, 0.1, 8, 3, 1, order=4), **W.airfoil_flow()),
    "ogrid_rotated": _rotated_ogrid,
}


@pytest.mark.parametrize("name", sorted(MESHES))
def test_neighbour_tables_bit_identical_to_oracle(name):
    m = MESHES[name]()
    m.setdefault("gamma", 1.4)
    nb_lib, x_lib = connectivity(m)
    o = OracleMesh(m)
    nb_orc = o.neighbours()
    assert nb_lib.dtype == nb_orc.dtype
    assert np.array_equal(nb_lib, nb_orc)
    assert np.abs(x_lib - o.solution_points()).max() < 1e-13
    # involution: partner of partner is self
    flat = nb_lib.ravel()
    inner = np.nonzero(flat >= 0)[0]
    assert np.array_equal(flat[flat[inner]], inner)


def test_unlisted_boundary_face_is_rejected():
    m = dict(W.naca_ogrid(0.04, 0.4, 0.12, 8, 3, 1), **W.airfoil_flow())
    m["bfaces"] = m["bfaces"][1:]
    with pytest.raises(_lib.FRError) as ei:
        connectivity(m)
    assert ei.value.code == _lib.FR_E_MESH


def test_inverted_element_is_rejected():
    m = W.box_mesh(2, (2, 2), (0, 0), (1, 1), order=2)
    en = m["elem_nodes"].copy()
    en[0] = en[0][[1, 0, 3, 2]]  # mirror: negative Jacobian
    m["elem_nodes"] = en
    with pytest.raises(_lib.FRError) as ei:
        connectivity(m)
    assert ei.value.code in (_lib.FR_E_MESH,)


def test_bad_node_id_is_rejected():
    m = W.box_mesh(2, (2, 2), (0, 0), (1, 1), order=2)
    m["elem_nodes"] = m["elem_nodes"].copy()
    m["elem_nodes"][1, 2] = 10 ** 6
    with pytest.raises(_lib.FRError) as ei:
        connectivity(m)
    assert ei.value.code == _lib.FR_E_ARG


def test_footprint_grows_with_mesh_and_precision():
    small = W.config_airfoil(0, ni=16, nj=4, nk=2)
    big = W.config_airfoil(0, ni=32, nj=8, nk=2)
    assert footprint(big, "fp32") > 3 * footprint(small, "fp32")
    assert footprint(small, "fp64") > footprint(small, "fp32")
