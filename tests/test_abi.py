"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, validates descriptions, and its host-built geometry and
covering-set index maps equal the oracle's bit for bit."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads
from oracle.geometry import Decomposition

pytestmark = pytest.mark.filterwarnings("ignore")


@pytest.fixture(scope="module")
def S():
    from paper_1710_02401_amd import swr
    if not os.path.exists(swr.LIB_PATH):
        pytest.fail("libswr.so is not built: run __graft_entry__.build() first")
    swr.load_library()
    return swr


def test_header_declarations_are_exported(S, repo_root):
    hdr = open(os.path.join(repo_root, "include", "swr.h")).read()
    declared = set(re.findall(r"\b(swr_[a-z_]+)\s*\(", hdr))
    lib = S.load_library()
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(S.EXPORTS)


TINY = {c["name"]: c for c in workloads.tiny_configs()}


def _create(S, cfg):
    d, keep = S.desc_from_config(cfg)
    h = ctypes.c_void_p()
    rc = S.load_library().swr_create(ctypes.byref(d), ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("mutate,code", [
    (dict(L=[0]), -1),
    (dict(overlap=[12.0]), -1),
    (dict(dt=0.0), -1),
    (dict(nbasis=[257]), -2),
    (dict(mode="tise", mu=[0.0, -1.0]), -1),
    (dict(mode="tise", mu=[1.0, 0.0], geometries=[[[0.0]], [[0.5]]]), -1),
    (dict(field=dict(E0=0.1, omega=1.0, phase=0.0, axis=3)), -1),
    (dict(learned_nodes=1), -1),
    (dict(learned_nodes=65), -1),
])
def test_invalid_descriptions_rejected(S, mutate, code):
    cfg = workloads.tiny_configs()[0]
    cfg.update(mutate)
    rc, h = _create(S, cfg)
    assert rc == code
    assert S.load_library().swr_last_error(None)


def test_factor_mode_validated_and_reported(S):
    lib = S.load_library()
    cfg = workloads.tiny_configs()[0]
    d, keep = S.desc_from_config(cfg)
    d.factor_mode = 4
    h = ctypes.c_void_p()
    assert lib.swr_create(ctypes.byref(d), ctypes.byref(h)) == -1
    assert b"factor_mode" in lib.swr_last_error(None)
    # the block path takes two or four configuration dimensions
    d.factor_mode = 3
    assert lib.swr_create(ctypes.byref(d), ctypes.byref(h)) == S.SWR_E_SIZE
    assert b"block path" in lib.swr_last_error(None)
    rc, h = _create(S, dict(cfg, factor="direct"))
    assert rc == 0
    info = S.swr_info()
    assert lib.swr_query(h, ctypes.byref(info)) == 0 and info.factor_terms == -1
    lib.swr_destroy(h)


def _circ(coords, **kw):
    f = dict(shape="circular", E0=1.0, omega=8.0, phase=0.0, nu=10.0, center=1.25,
             coords=coords, axis=0)
    f.update(kw)
    return f


@pytest.mark.parametrize("cfg_name,field,mode,ok,text", [
    ("paper-test-3", _circ([[0], [1]]), "tdse", True, None),
    ("c5-mini", _circ([[0, 2], [1, 3]]), "tdse", True, None),   # x.E of both electrons
    ("paper-test-3", _circ([[0], [0]]), "tdse", False, b"disjoint"),
    ("paper-test-3", _circ([[0, 1], []]), "tdse", False, b"disjoint"),
    ("paper-test-3", _circ([[0], [2]]), "tdse", False, b"disjoint"),
    ("paper-test-3", _circ([[0], [1]], nu=-1.0), "tdse", False, b"pulse_nu"),
    ("paper-test-2a", _circ([[0], [1]]), "tise", False, b"real time"),
])
def test_circular_field_validated(S, cfg_name, field, mode, ok, text):
    """The two-component field of Section 5, Test 3: masks within the
    configuration coordinates and disjoint, a non-negative envelope rate,
    real time only; a valid one inverts every step."""
    lib = S.load_library()
    cfg = workloads.get_config(cfg_name, field=field)
    assert cfg["mode"] == mode
    rc, h = _create(S, cfg)
    if not ok:
        assert rc == S.SWR_E_ARG and text in lib.swr_last_error(None)
        return
    assert rc == 0
    info = S.swr_info()
    assert lib.swr_query(h, ctypes.byref(info)) == 0 and info.wide == 0
    lib.swr_destroy(h)
    d, keep = S.desc_from_config(cfg)
    d.field_shape = 2
    h = ctypes.c_void_p()
    assert lib.swr_create(ctypes.byref(d), ctypes.byref(h)) == S.SWR_E_ARG
    assert b"field_shape" in lib.swr_last_error(None)


def test_second_dipole_only_for_circular_fields(S):
    """swr_get_matrix's Q2 (index 7) exists for a circular field only;
    indices past it are rejected (both before any device work)."""
    lib = S.load_library()
    rc, h = _create(S, workloads.tiny_configs()[0])
    assert rc == 0
    for which in (7, 8, -1):
        assert lib.swr_get_matrix(h, which, None, 0, None) == S.SWR_E_ARG
    lib.swr_destroy(h)


def test_random_small_configurations_accepted(S):
    """The seeded configurations of the GPU parity sweep are valid
    descriptions (checked here, on the CPU, before any GPU run)."""
    lib = S.load_library()
    for cfg in workloads.random_small_configs(10):
        rc, h = _create(S, cfg)
        assert rc == 0, (cfg["name"], lib.swr_last_error(None))
        lib.swr_destroy(h)


def test_unbound_workspace_and_state_errors(S):
    lib = S.load_library()
    rc, h = _create(S, workloads.tiny_configs()[0])
    assert rc == 0
    assert lib.swr_assemble(h, None) == S.SWR_E_STATE
    assert lib.swr_sweep(h, None) == S.SWR_E_STATE
    terms = np.zeros(64, dtype=np.int32)
    assert lib.swr_get_terms(h, terms.ctypes.data_as(S._c_i32p), terms.size) == S.SWR_E_STATE
    r = ctypes.c_double()
    assert lib.swr_transmit(h, ctypes.byref(r), None) == S.SWR_E_STATE
    # misaligned / too small workspace
    assert lib.swr_bind_workspace(h, ctypes.c_void_p(0x1001), 1 << 40) == S.SWR_E_ARG
    assert lib.swr_bind_workspace(h, ctypes.c_void_p(0x100000), 16) == S.SWR_E_SIZE
    lib.swr_destroy(h)


def _oracle_maps(dec):
    rows = []
    for s in dec.subs:
        for F in s.faces:
            for q in range(F.nodes.shape[0]):
                row = [-1] * 16
                if not F.is_global:
                    c = F.cover[q]
                    row[0] = len(c)
                    row[1:1 + len(c)] = [int(v) for v in c]
                rows.append(row)
    return np.array(rows, dtype=np.int32)


@pytest.mark.parametrize("name", ["tiny-1d", "tiny-2d", "c1-1e-1d", "c2-2e-1d", "tiny-slater",
                                  "c2-2e-1d-slater", "tiny-lsd", "paper-lsd-test-2a",
                                  "tiny-lsd-aug", "paper-lsd-test-2b", "tiny-lo"])
def test_index_maps_and_boxes_bit_exact(S, name):
    cfgs = {c["name"]: c for c in workloads.tiny_configs() + workloads.slater_configs()
            + workloads.lsd_configs() + workloads.lo_configs()}
    cfg = cfgs.get(name) or workloads.get_config(name)
    lib = S.load_library()
    rc, h = _create(S, cfg)
    assert rc == 0
    info = S.swr_info()
    assert lib.swr_query(h, ctypes.byref(info)) == 0
    dec = Decomposition(cfg)
    assert info.n_items == dec.n_sub
    bx = np.zeros(info.n_items * 8)
    assert lib.swr_get_boxes(h, bx.ctypes.data_as(S._c_f64p), bx.size) == 0
    bx = bx.reshape(-1, 4, 2)
    for s in dec.subs:
        for k in range(dec.D):
            assert bx[s.lin, k, 0] == s.lo[k] and bx[s.lin, k, 1] == s.hi[k]
    im = np.zeros(info.n_face_nodes * 16, dtype=np.int32)
    assert lib.swr_get_index_maps(h, im.ctypes.data_as(S._c_i32p), im.size) == 0
    assert np.array_equal(im.reshape(-1, 16), _oracle_maps(dec))
    # face nodes: independent Gauss-Legendre constructions agree to rounding
    x = np.zeros(info.n_face_nodes * 4)
    w = np.zeros(info.n_face_nodes)
    assert lib.swr_get_face_nodes(h, x.ctypes.data_as(S._c_f64p), w.ctypes.data_as(S._c_f64p),
                                  info.n_face_nodes) == 0
    xr = np.concatenate([F.nodes for s in dec.subs for F in s.faces])
    wr = np.concatenate([F.weights for s in dec.subs for F in s.faces])
    assert np.max(np.abs(x.reshape(-1, 4)[:, :dec.D] - xr)) < 1e-14
    assert np.max(np.abs(w - wr)) < 1e-14
    # items: sizes and multi-indices
    it = np.zeros(info.n_items * 10, dtype=np.int32)
    assert lib.swr_get_items(h, it.ctypes.data_as(S._c_i32p), it.size) == 0
    it = it.reshape(-1, 10)
    for s in dec.subs:
        assert it[s.lin, 0] == s.K
        assert tuple(it[s.lin, 2:2 + dec.D]) == s.idx
        assert tuple(it[s.lin, 6:6 + dec.D]) == s.nb
    lib.swr_destroy(h)


@pytest.mark.parametrize("M,cases", [
    (0, [(8, False), (10, False), (11, True), (200, True), (1000, True)]),
    (16, [(45, False), (46, True), (200, True)]),
    (32, [(190, False), (195, True), (1000, True)]),
    (64, [(1000, True)]),
])
def test_time_nodes_match_oracle_and_short_windows_are_rejected(S, M, cases):
    from oracle import learned as o_learned
    lib = S.load_library()
    for n_steps, ok in cases:
        cfg = dict(workloads.tiny_configs()[1], n_steps=n_steps, learned_nodes=M)
        rc, h = _create(S, cfg)
        assert rc == 0
        info = S.swr_info()
        assert lib.swr_query(h, ctypes.byref(info)) == 0
        assert info.learned_nodes == (M or 8)
        out = np.zeros(info.learned_nodes, dtype=np.int32)
        rc = lib.swr_time_nodes(h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        if ok:
            assert rc == 0 and list(out) == o_learned.time_nodes(n_steps, M or 8)
        else:
            assert rc == -1 and b"not distinct" in lib.swr_last_error(h)
            with pytest.raises(ValueError):
                o_learned.time_nodes(n_steps, M or 8)
        lib.swr_destroy(h)


def test_batched_geometries_share_one_decomposition(S):
    """Items are geometry-major copies of one decomposition: per-item sizes
    repeat per geometry and the covering sets stay inside a geometry."""
    cfg = workloads.get_config("c3-mini")
    rc, h = _create(S, cfg)
    assert rc == 0
    lib = S.load_library()
    n_sub, n_geom = 16, 4
    items = np.zeros(n_sub * n_geom * 10, dtype=np.int32)
    assert lib.swr_get_items(h, items.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), items.size) == 0
    K = items.reshape(-1, 10)[:, 0]
    assert list(K) == [nb[0] for nb in cfg["nbasis"]] * n_geom
    info = S.swr_info()
    assert lib.swr_query(h, ctypes.byref(info)) == 0
    maps = np.zeros(info.n_face_nodes * 16, dtype=np.int32)
    assert lib.swr_get_index_maps(h, maps.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), maps.size) == 0
    maps = maps.reshape(-1, 16)
    per_geom = maps.shape[0] // n_geom
    assert np.array_equal(maps[:per_geom], maps[per_geom:2 * per_geom])
    dec = Decomposition(dict(cfg, nuclei=cfg["geometries"][0]))
    assert np.array_equal(maps[:per_geom], _oracle_maps(dec))
    lib.swr_destroy(h)


def test_local_orbital_basis_in_two_dimensions_is_validated(S):
    """Local orbitals of one electron in two dimensions (Section 3, d = 2)
    take one electron in two dimensions, 1..(Gaussians per box) orbitals, at
    most 8 Gaussians per dimension, positive barrier and mollifier widths, a
    mollifier order of at least 2, no added Gaussians and one geometry."""
    lib = S.load_library()
    base = workloads.lo_configs()[0]
    rc, h = _create(S, base)
    assert rc == 0
    info = S.swr_info()
    assert lib.swr_query(h, ctypes.byref(info)) == 0 and info.K_max == 8 and info.tx_tile == 0
    lib.swr_destroy(h)
    bad_lo = [(dict(orbitals=0), "lsd_orbitals"), (dict(orbitals=26), "lsd_orbitals"),
              (dict(moll_order=1), "lsd_moll_order"), (dict(moll_eps=0.0), "lsd_moll_eps"),
              (dict(augment=1), "lsd_augment")]
    for bad, why in bad_lo:
        rc, h = _create(S, dict(base, lo=dict(base["lo"], **bad)))
        assert rc == S.SWR_E_ARG, bad
        assert why in lib.swr_last_error(None).decode(), bad
    for bad, why in [(dict(nbasis=[9, 5]), "8 Gaussians"),
                     (dict(n_elec=2, dim=1, nuclei=[[0.3]]), "one electron in two dimensions")]:
        rc, h = _create(S, dict(base, **bad))
        assert rc == S.SWR_E_ARG, bad
        assert why in lib.swr_last_error(None).decode(), bad


def test_schedule_is_set_only_after_assembly(S):
    """swr_set_schedule needs the assembled problem (SWR_E_STATE before
    swr_assemble, checked without a device) and a handle (SWR_E_ARG)."""
    lib = S.load_library()
    rc, h = _create(S, workloads.tiny_configs()[0])
    assert rc == 0
    assert lib.swr_set_schedule(h, 1, 16, 0, None) == S.SWR_E_STATE
    assert "swr_assemble" in lib.swr_last_error(h).decode()
    assert lib.swr_set_schedule(None, 1, 16, 0, None) == S.SWR_E_ARG
    lib.swr_destroy(h)


def test_wide_bases_take_the_wide_path(S):
    """One electron in one dimension (real time) accepts up to 256 Gaussians
    per subdomain on the wide-basis path: the full batched workload (64
    geometries x 256 subdomains, K = 32..256) is created with depth 1 and no
    per-step inverses in its workspace; the path can also be asked for at
    K <= 64, and is refused elsewhere."""
    lib = S.load_library()
    cfg = workloads.get_config("c3-1e-1d-batched")
    rc, h = _create(S, cfg)
    assert rc == 0
    info = S.swr_info()
    assert lib.swr_query(h, ctypes.byref(info)) == 0
    assert info.wide == 1 and info.K_max == 256 and info.n_items == 64 * 256
    # one iterate at a time; the wide transmission's default tile (16 steps)
    # and recurrence order (largest K first) until swr_autotune chooses
    assert info.depth == 1 and info.tx_tile == 16 and info.wide_order == 0 and info.tuned == 0
    # matrices, series terms and histories, far below one inverse per step
    # (200 x sum K^2 x 16 bytes)
    assert info.workspace_bytes < 200 * info.sum_K2 * 16 / 4
    lib.swr_destroy(h)
    rc, h = _create(S, workloads.get_config("c1-1e-1d"))
    info = S.swr_info()
    assert rc == 0 and lib.swr_query(h, ctypes.byref(info)) == 0 and info.wide == 0
    lib.swr_destroy(h)
    rc, h = _create(S, dict(workloads.get_config("c1-1e-1d"), factor="wide"))
    assert rc == 0 and lib.swr_query(h, ctypes.byref(info)) == 0 and info.wide == 1
    lib.swr_destroy(h)


@pytest.mark.parametrize("mutate,code,text", [
    (dict(nbasis=[9, 9]), -2, b"exceeds 64"),
    (dict(factor="wide"), -1, b"wide-basis path"),
])
def test_wide_bases_refused_beyond_one_dimension(S, mutate, code, text):
    cfg = [c for c in workloads.tiny_configs() if c["name"] == "tiny-2d"][0]
    rc, h = _create(S, dict(cfg, **mutate))
    assert rc == code
    assert text in S.load_library().swr_last_error(None)


@pytest.mark.parametrize("mutate", [dict(factor="direct"), dict(mu=[0.0, 1.0])])
def test_wide_bases_need_the_series(S, mutate):
    cfg = dict(workloads.get_config("c3-wide"), **mutate)
    rc, h = _create(S, cfg)
    assert rc == -2
    assert b"field series" in S.load_library().swr_last_error(None)


def test_slater_basis_needs_an_exchange_symmetric_two_electron_problem(S):
    """The Slater-like basis (Section 2, eq. (LSD)) is for two electrons in
    one dimension each on a decomposition symmetric under their exchange;
    every other description is refused with the reason."""
    lib = S.load_library()
    base = workloads.slater_configs()[0]
    rc, h = _create(S, base)
    assert rc == 0
    lib.swr_destroy(h)
    for bad, why in [(dict(L=[3, 2]), "symmetric"), (dict(nbasis=[4, 3]), "one basis size"),
                     (dict(overlap=[0.8, 0.7]), "symmetric"),
                     (dict(factor="wide"), "narrow path"),
                     (dict(init=dict(alpha=0.6, center=[0.5, 0.5])), "distinct centres")]:
        rc, h = _create(S, dict(base, **bad))
        assert rc == S.SWR_E_ARG, bad
        assert why in lib.swr_last_error(None).decode(), bad
    one = dict(TINY["tiny-1d"], basis="slater")
    rc, h = _create(S, one)
    assert rc == S.SWR_E_ARG and "two electrons" in lib.swr_last_error(None).decode()


def test_local_orbital_parameters_are_validated(S):
    """Local Slater determinants (Section 3) take 2..8 orbitals, at most the
    Gaussians per interval, positive barrier and mollifier widths, at most 8
    functions and at most the Gaussians per interval with the added end
    Gaussians (Section 3.3), and the Slater basis's conditions on the
    problem."""
    lib = S.load_library()
    base = workloads.lsd_configs()[0]
    rc, h = _create(S, base)
    assert rc == 0
    lib.swr_destroy(h)
    for bad, why in [(dict(orbitals=1), "lsd_orbitals"), (dict(orbitals=7), "lsd_orbitals"),
                     (dict(moll_eps=0.0), "lsd_moll_eps"), (dict(barrier_width=-1.0), "lsd_barrier"),
                     (dict(moll_order=0), "lsd_moll_order"), (dict(augment=-1), "lsd_augment"),
                     (dict(augment=2), "lsd_augment"), (dict(orbitals=5, augment=1), "lsd_augment")]:
        rc, h = _create(S, dict(base, lsd=dict(base["lsd"], **bad)))
        assert rc == S.SWR_E_ARG, bad
        assert why in lib.swr_last_error(None).decode(), bad
    rc, h = _create(S, dict(base, L=[3, 2]))
    assert rc == S.SWR_E_ARG and "symmetric" in lib.swr_last_error(None).decode()


@pytest.mark.parametrize("name,extra", [("tiny-1d", {}), ("tiny-2d", {}),
                                        ("tiny-2d", {"factor": "block"})])
def test_singular_gram_refused(S, name, extra):
    """Gaussians 30 wide on subdomains a few units across are linearly
    dependent to working precision (their Gram matrix's Cholesky
    factorisation fails): swr_create returns SWR_E_SINGULAR on the narrow
    and the block path alike, naming the cause; the same boxes at their
    workload's widths are accepted."""
    cfg = dict(TINY[name], width=30.0, width_ratio=None, **extra)
    rc, h = _create(S, cfg)
    assert rc == S.SWR_E_SINGULAR
    msg = S.load_library().swr_last_error(None).decode()
    assert "singular to working precision" in msg
    rc, h = _create(S, dict(TINY[name], **extra))
    assert rc == 0
    S.load_library().swr_destroy(h)


def test_ill_conditioned_gram_refused(S):
    """The paper's Test 3 boxes with Test 2.a's delta = 0.5 make the Gram
    matrices nearly singular (condition 1.6e8): swr_create refuses them with
    SWR_E_COND instead of running a recurrence whose stored inverses would
    put the answer measurably off; the same boxes with widths 0.7 x spacing
    (condition 2.2e3) are accepted."""
    cfg = workloads.get_config("paper-test-3", width=1.0, width_ratio=None)
    rc, h = _create(S, cfg)
    assert rc == S.SWR_E_COND
    msg = S.load_library().swr_last_error(None).decode()
    assert "condition" in msg and "1.6" in msg
    rc, h = _create(S, workloads.get_config("paper-test-3"))
    assert rc == 0
    S.load_library().swr_destroy(h)
