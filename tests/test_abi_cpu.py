"""CPU-only tests of the C ABI: the library loads, exports every declared symbol,
validates configurations, reports errors without a GPU, and its host balancer
gives bit-identical maps to the oracle's."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_1310_4218_amd import _abi, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbgrid.h")


@pytest.fixture(scope="session")
def lib():
    if not os.path.exists(_abi.LIB_PATH):
        from paper_1310_4218_amd import build_lib
        build_lib.build()
    return _abi.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(lb_\w+)\s*\(", text, flags=re.M)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_abi.SIGNATURES), "binding and header disagree"


def test_struct_layout_and_version(lib):
    assert lib.lb_abi_version() == 7
    assert lib.lb_config_bytes() == C.sizeof(_abi.LbConfig)
    assert lib.lb_stats_bytes() == C.sizeof(_abi.LbStats)


def test_query_sizes(lib):
    wl = W.small()
    cfg, keep = _abi.config_from_workload(wl)
    b = _abi.query(cfg)
    assert b[0] == b[1] == 64 * 64 * 32 * 4
    cfg64, keep = _abi.config_from_workload(wl, precision="fp64", nfields=3)
    b64 = _abi.query(cfg64)
    assert b64[0] == 3 * 64 * 64 * 32 * 8
    assert b[2] > 0 and b[2] % 256 == 0


@pytest.mark.parametrize("field,value,msg", [
    ("nx", 0, "nx"), ("nz", 0, "nz"), ("px", 65, "px"), ("precision", 7, "precision"),
    ("nslots", 0, "nslots"), ("kmax", 0, "kmin"), ("nhot", 5, "nhot"), ("graph_steps", 0, "graph"),
    ("steal", 2, "steal"), ("nfields", 0, "nfields"), ("sigma", -1.0, "sigma"),
    ("tile_x", 2000, "1024"), ("alpha_work", -1, "alpha"), ("wg_per_queue", 100000, "65536"),
    ("item_alpha", -2, "item_alpha"),
])
def test_query_rejects_bad_config(lib, field, value, msg):
    cfg, keep = _abi.config_from_workload(W.small())
    setattr(cfg, field, value)
    b = _abi.LbBuffers()
    rc = lib.lb_query(C.byref(cfg), C.byref(b))
    assert rc == _abi.LB_E_INVAL
    assert msg in lib.lb_last_error(None).decode()


@pytest.mark.parametrize("over,msg", [
    (dict(stage_rows=-3), "stage_rows"), (dict(stage_rows=-16), "stage_rows"),
    (dict(stage_rows=33), "stage_rows"), (dict(stage_rows=-8, precision=2), "FP32 only"),
    (dict(stage_rows=-4, nz=6), "divisible by 4"), (dict(stage_rows=2, nz=6), "divisible by 4"),
    (dict(stage_rows=-4, tile_x=80), "512 threads"),
    (dict(stage_rows=-1, precision=2, tile_x=80), "FP64"),
    (dict(march=3), "march must be"), (dict(march=2, nz=6), "march needs nz divisible by 4"),
    (dict(march=4, precision=2, tile_x=70), "FP64 march"), (dict(march=8, tile_x=200), "1024 threads"),
    (dict(item_grid=1), "item_grid needs the column-march"), (dict(item_grid=2, march=2), "item_grid must be"),
    (dict(queue_order=3), "queue_order must be"), (dict(hot_cut=-1), "hot_cut"),
    (dict(fuse_steps=4), "fuse_steps must be"), (dict(fuse_steps=2, march=2), "fuse_steps 2 or 3 needs item_grid"),
    (dict(fuse_steps=3, march=2), "fuse_steps 2 or 3 needs item_grid"),
    (dict(fuse_steps=3, march=2, item_grid=1, precision=2, tile_x=59), "fuse_steps 3 in FP64"),
    (dict(fuse_steps=2, march=2, item_grid=1, precision=2, tile_x=61), "fuse_steps 2 in FP64"),
    (dict(fuse_steps=2, march=2, item_grid=1, tile_x=125), "fuse_steps 2 needs (tile_x + 4)"),
    (dict(lane_levels=3), "lane_levels must be"),
    (dict(xcd_group=65, march=2, item_grid=1), "xcd_group must be"),
    (dict(xcd_group=-1), "xcd_group must be"), (dict(xcd_group=4, march=2), "xcd_group needs item_grid 1"),
    (dict(lane_levels=5, march=2, item_grid=1), "lane_levels 5 needs fuse_steps 2"),
    (dict(lane_levels=5, march=2, item_grid=1, fuse_steps=3), "lane_levels 5 needs fuse_steps 2"),
    (dict(lane_levels=5, march=2, item_grid=1, fuse_steps=2), "nz divisible by 20"),
    (dict(lane_levels=5, march=8, item_grid=1, fuse_steps=2, nz=40), "march 2 or 4"),
])
def test_query_rejects_bad_pipeline(lib, over, msg):
    """Register pipeline depths are 2, 4 or 8 rows; the deep ones need V = 4 and
    workgroups of at most 512 threads, and depth 8 is FP32 only.  The column march
    takes 2, 4 or 8 rows in flight, needs V = 4 and (tile_x + 2) * nz / 4 threads, at
    most 512 in FP64; two steps per launch need item_grid 1 and (tile_x + 4) * nz / 4
    threads, three steps (tile_x + 6) * nz / 4.  (64x64x32: tile_x 61 and 125 fit one step
    per launch but not two; tile_x 59 fits two in FP64 but not three.)  Five levels per
    thread (lane_levels 5) is for the two-step launch only, with nz % 20 == 0 and 2 or 4
    rows in flight."""
    cfg, keep = _abi.config_from_workload(W.small())
    for k, v in over.items():
        setattr(cfg, k, v)
    b = _abi.LbBuffers()
    assert lib.lb_query(C.byref(cfg), C.byref(b)) == _abi.LB_E_INVAL
    assert msg in lib.lb_last_error(None).decode()


def test_vertical_layouts(lib):
    """Vertical physics passes levels up a column's lanes inside one wave: columns of lanes
    that do not divide 64 (80 levels: 20 lanes) need the march, which lays out whole columns
    per wave; more than 64 lanes per column are never possible."""
    from paper_1310_4218_amd._abi import LbError
    wl = W.small().replace(nz=80, vertical=1)
    with pytest.raises(LbError) as e:
        _abi.query(_abi.config_from_workload(wl)[0])
    assert e.value.code == _abi.LB_E_UNSUPPORTED
    _abi.query(_abi.config_from_workload(wl, march=2)[0])
    _abi.query(_abi.config_from_workload(wl, march=4, item_grid=1, tile_x=14)[0])
    _abi.query(_abi.config_from_workload(wl, march=4, item_grid=1, fuse_steps=2, tile_x=14)[0])
    with pytest.raises(LbError) as e:
        _abi.query(_abi.config_from_workload(W.small().replace(nz=260, vertical=1), march=2)[0])
    assert e.value.code == _abi.LB_E_UNSUPPORTED


def test_measure_halves_need_a_context(lib):
    assert lib.lb_measure_begin(None, 0, 1) == _abi.LB_E_INVAL
    assert lib.lb_measure_end(None, None) == _abi.LB_E_INVAL
    assert lib.lb_field_sum_noalloc(None, 0, 10, None, None) == _abi.LB_E_INVAL


def test_query_accepts_pipeline_depths(lib):
    for over in (dict(stage_rows=-1), dict(stage_rows=-2), dict(stage_rows=-4),
                 dict(stage_rows=-8), dict(stage_rows=-4, precision=2), dict(stage_rows=6)):
        cfg, keep = _abi.config_from_workload(W.small())
        for k, v in over.items():
            setattr(cfg, k, v)
        b = _abi.LbBuffers()
        assert lib.lb_query(C.byref(cfg), C.byref(b)) == _abi.LB_OK, over


def test_query_rejects_bad_splits(lib):
    for xs in ([0, 10, 10, 64], [0, 20, 40, 63], [1, 20, 40, 64], [0, 30, 20, 64]):
        cfg, keep = _abi.make_config(64, 64, 8, 3, 1, xs, [0, 64])
        b = _abi.LbBuffers()
        assert lib.lb_query(C.byref(cfg), C.byref(b)) == _abi.LB_E_INVAL
        assert "xsplit" in lib.lb_last_error(None).decode()


def test_init_argument_errors_without_gpu(lib):
    cfg, keep = _abi.config_from_workload(W.small())
    sizes = _abi.query(cfg)
    h = C.c_void_p()
    b = _abi.LbBuffers()
    assert lib.lb_grid_init(C.byref(cfg), C.byref(b), None, None, C.byref(h)) == _abi.LB_E_INVAL
    assert h.value is None
    for i in range(3):                      # fake, aligned, never dereferenced
        b.ptr[i] = 0x100000 * (i + 1)
        b.bytes[i] = sizes[i]
    b.bytes[2] = sizes[2] - 8
    assert lib.lb_grid_init(C.byref(cfg), C.byref(b), None, None, C.byref(h)) == _abi.LB_E_NOMEM
    assert "too small" in lib.lb_last_error(None).decode()
    b.bytes[2] = sizes[2]
    b.ptr[1] = 0x100010
    assert lib.lb_grid_init(C.byref(cfg), C.byref(b), None, None, C.byref(h)) == _abi.LB_E_INVAL
    assert "aligned" in lib.lb_last_error(None).decode()
    b.ptr[1] = 0x200000
    os.environ["LBGRID_FAIL_AT"] = "init"
    try:
        assert lib.lb_grid_init(C.byref(cfg), C.byref(b), None, None, C.byref(h)) == _abi.LB_E_HIP
        assert "forced" in lib.lb_last_error(None).decode()
    finally:
        del os.environ["LBGRID_FAIL_AT"]


def test_null_context_calls(lib):
    assert lib.lb_step(None, 1, 1) == _abi.LB_E_INVAL
    assert lib.lb_measure(None, 0, None, 0) == _abi.LB_E_INVAL
    assert lib.lb_rebalance(None, 0, 1.0, None, None, None, None) == _abi.LB_E_INVAL
    assert lib.lb_fields(None, 0, None, 0, None) == _abi.LB_E_INVAL
    assert lib.lb_set_map(None, None, None) == _abi.LB_E_INVAL
    lib.lb_destroy(None)


def random_loads(rng, C_):
    kind = rng.integers(0, 3)
    if kind == 0:
        return rng.integers(1, 8, size=C_).astype(float)           # many ties
    if kind == 1:
        return np.round(rng.uniform(0, 1e6, size=C_))
    return rng.uniform(0.0, 5.0, size=C_)


def test_host_greedy_bit_exact_vs_oracle(lib):
    rng = np.random.default_rng(1)
    for _ in range(300):
        C_ = int(rng.integers(0, 300))
        S = int(rng.integers(1, 40))
        w = random_loads(rng, C_)
        m, nm = _abi.balance_host(w, S, "greedy")
        ref = oracle.greedy(w, S)
        np.testing.assert_array_equal(m, ref)
        assert nm == int((ref != oracle.block_map(C_, S)).sum())


def test_host_refine_bit_exact_vs_oracle(lib):
    rng = np.random.default_rng(2)
    for _ in range(300):
        C_ = int(rng.integers(1, 300))
        S = int(rng.integers(1, 40))
        w = random_loads(rng, C_)
        old = rng.integers(0, S, size=C_).astype(np.int32)
        for thr in (1.0, 1.05, 1.2):
            m, nm = _abi.balance_host(w, S, "refine", old_map=old, threshold=thr)
            ref = oracle.refine(w, old, S, thr)
            np.testing.assert_array_equal(m, ref)
            assert nm == int((ref != old).sum())


def test_host_refineswap_bit_exact_vs_oracle(lib):
    rng = np.random.default_rng(3)
    for _ in range(300):
        C_ = int(rng.integers(1, 200))
        S = int(rng.integers(1, 30))
        w = random_loads(rng, C_)
        old = rng.integers(0, S, size=C_).astype(np.int32)
        for thr in (1.0, 1.05, 1.2):
            m, nm = _abi.balance_host(w, S, "refineswap", old_map=old, threshold=thr)
            ref = oracle.refineswap(w, old, S, thr)
            np.testing.assert_array_equal(m, ref)
            assert nm == int((ref != old).sum())


def test_host_greedy_then_refineswap_vs_oracle(lib):
    """Strategy 3 is Greedy on a first call (no old map) and RefineSwap from the old map
    otherwise, bit-exact against the oracle's policy."""
    rng = np.random.default_rng(4)
    for _ in range(150):
        C_ = int(rng.integers(1, 200))
        S = int(rng.integers(1, 30))
        w = random_loads(rng, C_)
        m, nm = _abi.balance_host(w, S, "greedy_then_refineswap")
        ref = oracle.greedy_then_refineswap(w, None, S, 1.05, first=True)
        np.testing.assert_array_equal(m, ref)
        assert nm == int((ref != oracle.block_map(C_, S)).sum())
        old = rng.integers(0, S, size=C_).astype(np.int32)
        for thr in (1.0, 1.05):
            m, nm = _abi.balance_host(w, S, "greedy_then_refineswap", old_map=old, threshold=thr)
            ref = oracle.greedy_then_refineswap(w, old, S, thr, first=False)
            np.testing.assert_array_equal(m, ref)
            assert nm == int((ref != old).sum())


def test_host_balancer_large_instance(lib):
    wl = W.large()
    k = oracle.kfield(wl.nx, wl.ny, wl.hot, 0, wl.sigma, wl.kmin, wl.kmax)
    w = oracle.chunk_work(k, wl.nz, wl.xsplit, wl.ysplit, wl.alpha_work)
    m, _ = _abi.balance_host(w, 256, "greedy")
    np.testing.assert_array_equal(m, oracle.greedy(w, 256))
    old = oracle.block_map(len(w), 256)
    m, _ = _abi.balance_host(w, 256, "refine", old_map=old, threshold=1.05)
    np.testing.assert_array_equal(m, oracle.refine(w, old, 256, 1.05))


def test_host_balancer_errors(lib):
    w = np.ones(4)
    with pytest.raises(_abi.LbError):
        _abi.balance_host(np.array([1.0, -1.0]), 2)
    with pytest.raises(_abi.LbError):
        _abi.balance_host(np.array([1.0, np.nan]), 2)
    with pytest.raises(_abi.LbError):
        _abi.balance_host(w, 0)
    with pytest.raises(_abi.LbError):
        _abi.balance_host(w, 2, "refine")                       # needs an old map
    with pytest.raises(_abi.LbError):
        _abi.balance_host(w, 2, "refine", old_map=[0, 1, 2, 0])  # slot out of range
    with pytest.raises(_abi.LbError):
        _abi.balance_host(w, 2, "refine", old_map=[0, 1, 1, 0], threshold=0.0)
