"""The C ABI library loads and exports every symbol the header declares.

No compute call is made: only entry points that return before touching the
GPU (argument validation, defaults, status strings).
"""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "maspncg.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:mas_status|void|const char\s*\*)\s*(\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def L():
    from paper_2604_19892_amd import _abi
    return _abi.lib()


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for n in ("mas_build", "mas_woodbury_update", "mas_apply", "hess_vec", "pncg_subspace_step"):
        assert n in names
    assert len(names) == 34


def test_every_declared_symbol_is_exported(L):
    for n in declared_functions():
        assert hasattr(L, n), n
    from paper_2604_19892_amd import _abi
    assert set(declared_functions()) == set(_abi.SIGNATURES)


def test_struct_layouts_match_header(L):
    from paper_2604_19892_amd import _abi
    # field order / sizes as in the header (8-byte aligned members)
    assert ctypes.sizeof(_abi.MasConfig) == 4 + 4 + 7 * 8 + 3 * 8 + 4 * 4 + 8 + 3 * 8 + 4 + 4  # precond, hierarchy
    assert ctypes.sizeof(_abi.MasIterStats) == 7 * 8 + 2 * 4 + 8 + 8 * 8
    assert ctypes.sizeof(_abi.MasMesh) == 2 * 8 + 5 * 8 + 2 * 8 + 8 + 8
    assert ctypes.sizeof(_abi.MasContacts) == 5 * 8
    assert ctypes.sizeof(_abi.MasStepOut) == 11 * 8 + 4 * 4


def test_default_config_holds_the_paper_constants(L):
    from paper_2604_19892_amd import _abi
    golden = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "paper_constants.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()[:2]
            golden[k] = float(v)
    cfg = _abi.MasConfig()
    L.mas_default_config(ctypes.byref(cfg))
    assert cfg.max_rank == golden["topk_K"]
    assert cfg.restart_delta == golden["restart_delta"]
    assert cfg.eps_sing == golden["eps_sing"]
    assert cfg.cos_rot == pytest.approx(np.cos(np.deg2rad(golden["rotation_threshold_deg"])), rel=1e-15)
    assert cfg.num_levels <= golden["max_levels"]


def test_argument_errors_return_without_gpu(L):
    from paper_2604_19892_amd import _abi
    cfg = _abi.MasConfig()
    L.mas_default_config(ctypes.byref(cfg))
    h = ctypes.c_void_p()
    assert L.mas_create(None, None, None, ctypes.byref(h), None) == 1
    mesh = _abi.MasMesh()
    mesh.num_vertices = 0
    assert L.mas_create(ctypes.byref(cfg), ctypes.byref(mesh), None, ctypes.byref(h), None) == 1
    cfg.num_levels = 9
    mesh.num_vertices = 4
    assert L.mas_create(ctypes.byref(cfg), ctypes.byref(mesh), None, ctypes.byref(h), None) == 1
    assert L.mas_apply(None, None, None) == 1
    assert L.hess_vec(None, None, None, 0) == 1
    assert L.mas_build(None, None, None) == 1
    assert L.mas_ccd_steps(None, None, None, 0, None, None, None, None, None) == 1
    assert L.mas_contact_distances(None, None, 0, None, None, None, None, None) == 1
    assert L.mas_constraint_set(None, None, 1e-3, 0, None, 0, None, 0, None, 0, None, None, None, None, None,
                                None) == 1
    assert L.mas_status_string(5) == b"non-positive pivot (matrix not SPD)"


@pytest.mark.parametrize("scene,levels", [("grid", 2), ("combs", 2), ("combs", 3), ("two_boxes", 3)])
def test_vertex_order_matches_oracle(L, scene, levels):
    """mas_vertex_order (host logic) against the oracle's orders, bit for
    bit: Morton and the connectivity-aware hierarchy."""
    from oracle import mas
    from paper_2604_19892_amd import synth
    from paper_2604_19892_amd.binding import vertex_order
    sc = {"grid": synth.grid_scene, "combs": synth.combs_scene, "two_boxes": synth.two_boxes_scene}[scene]()
    np.testing.assert_array_equal(vertex_order(sc.X, sc.tets, levels, "morton"), mas.morton_perm(sc.X))
    np.testing.assert_array_equal(vertex_order(sc.X, sc.tets, levels, "connectivity"),
                                  mas.connectivity_perm(sc.X, sc.tets, levels))
    links = synth.contact_links(sc.pool, sc.x, sc.dhat)
    np.testing.assert_array_equal(vertex_order(sc.X, sc.tets, levels, "connectivity", links),
                                  mas.connectivity_perm(sc.X, sc.tets, levels, links=links))


def test_vertex_order_rejects_bad_input(L):
    from paper_2604_19892_amd import _abi
    from paper_2604_19892_amd.binding import vertex_order
    X = np.zeros((4, 3))
    with pytest.raises(_abi.MasError):
        vertex_order(X, np.array([[0, 1, 2, 4]]), 1, "connectivity")
    with pytest.raises(_abi.MasError):
        vertex_order(X, np.array([[0, 1, 2, 3]]), 7, "connectivity")
    with pytest.raises(_abi.MasError):
        vertex_order(X, np.array([[0, 1, 2, 3]]), 1, "connectivity", links=np.array([[0, 4]]))
