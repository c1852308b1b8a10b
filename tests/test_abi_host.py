"""CPU checks of the C-ABI library: it loads, exports every declared symbol, validates its inputs,
and its host-side plan (cluster tree, block partition, element-pair classification; Sec. 4.1,
Sec. 4.2 Def., Sec. 4 item 4) is identical to the oracle's.  No GPU work is started here."""
import math
import os
import re

import numpy as np
import pytest

import oracle
from paper_1708_09162_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

igb = pytest.importorskip("paper_1708_09162_amd.igabem", reason="libigabem.so not built")


def test_library_exports_every_declared_symbol():
    with open(os.path.join(ROOT, "include", "igabem.h")) as fh:
        hdr = fh.read()
    declared = set(re.findall(r"\b(igb_[A-Za-z_0-9]+)\s*\(", hdr))
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(igb._lib, name), name
    assert declared == set(igb.EXPORTED)


def test_stage_names_match_header():
    with open(os.path.join(ROOT, "include", "igabem.h")) as fh:
        n = int(re.search(r"#define IGB_NUM_MATVEC_STAGES (\d+)", fh.read()).group(1))
    assert n == len(igb.STAGES)


def test_release_cached_memory_with_nothing_cached():
    # no operator was ever created in this process: nothing is cached and no HIP call is made
    igb.igb_release_cached_memory()
    igb.igb_release_cached_memory()


def test_single_precision_far_field_accepted_where_supported():
    g = igb.Geometry(W.sphere_patches())
    igb.Plan(g, p=1, m=2, q=8, mode=igb.IGB_H2_ONTHEFLY, far_precision=igb.IGB_FP32)


def test_geometry_validation_errors():
    good = W.sphere_patches()[0]
    igb.Geometry([good])
    bad_w = dict(good, cpw=good["cpw"].copy())
    bad_w["cpw"][0, 0, 3] = 0.0
    bad_knots = dict(good, knots_u=np.array([0, 0, 0, 0, 0.1, 1, 1, 1, 1, 1.0]))
    dec_knots = dict(good, knots_u=np.array([0, 0, 0, 0, 0, 1, 1, 1, 0.9, 1.0]))
    nan_cp = dict(good, cpw=good["cpw"].copy())
    nan_cp["cpw"][1, 1, 0] = np.nan
    for bad in (bad_w, bad_knots, dec_knots, nan_cp):
        with pytest.raises(igb.IgbError) as e:
            igb.Geometry([bad])
        assert e.value.status == igb.IGB_EINVAL
    with pytest.raises(igb.IgbError):
        igb.Geometry([])


@pytest.mark.parametrize("bad", [dict(p=-1), dict(p=7), dict(m=11), dict(q=0), dict(eta=0.0), dict(eta=-1.0),
                                 dict(gauss_regular=0), dict(gauss_singular=41), dict(kernel=5), dict(mode=3),
                                 dict(kernel=1, wavenumber=-1.0), dict(leaf_depth=-2), dict(far_precision=2),
                                 dict(far_precision=1, kernel=1, wavenumber=1.0, mode=2, q=11),
                                 dict(far_precision=1, mode=1), dict(far_precision=1, mode=2, q=9),
                                 dict(kernel=1, wavenumber=1e6), dict(kappa_diam=-1.0),
                                 dict(kappa_diam=float("inf"))])
def test_parameter_validation_errors(bad):
    g = igb.Geometry(W.sphere_patches())
    with pytest.raises(igb.IgbError) as e:
        igb.Plan(g, **bad)
    assert e.value.status == igb.IGB_EINVAL


def test_interior_knots_must_lie_on_refinement_grid():
    sq = W.flat_patch((0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0))
    # degree-1 patch with an interior knot at 1/3: fine at no refinement level with h = 2^-m
    p = dict(sq, knots_u=np.array([0, 0, 1 / 3, 1, 1.0]),
             cpw=np.stack([sq["cpw"][:, 0], (2 * sq["cpw"][:, 0] + sq["cpw"][:, 1]) / 3, sq["cpw"][:, 1]], axis=1))
    g = igb.Geometry([p])
    with pytest.raises(igb.IgbError) as e:
        igb.Plan(g, p=0, m=2, q=1)
    assert e.value.status == igb.IGB_EINVAL
    # a knot at 1/2 is on the grid for m >= 1
    p2 = dict(p, knots_u=np.array([0, 0, 0.5, 1, 1.0]))
    igb.Plan(igb.Geometry([p2]), p=0, m=1, q=1)


def _compare_plan(patches, **prm):
    dense = prm.pop("dense", False)
    g = igb.Geometry(patches)
    pl = igb.Plan(g, mode=igb.IGB_DENSE if dense else igb.IGB_H2_STORED, **prm)
    kw = dict(p=prm.get("p", 1), m=prm.get("m", 2), q=prm.get("q", 8), eta=1e-12 if dense else prm.get("eta", 1.6),
              leaf_depth=prm.get("leaf_depth", -1), gauss_regular=prm.get("gauss_regular", 6),
              kernel=prm.get("kernel", 0), wavenumber=prm.get("wavenumber", 0.0),
              kappa_diam=prm.get("kappa_diam", 0.0))
    P = oracle.Problem(patches, **kw)
    info = pl.info
    assert info.n_dof == P.ndof and info.n_dof_super == P.nsup and info.leaf_level == P.L
    near, far = pl.partition()
    onear, ofar = P.partition()
    assert np.array_equal(near, onear)
    assert np.array_equal(far, ofar)
    pairs = pl.pair_classes()
    opairs = P.near_pair_classes()
    assert np.array_equal(pairs, opairs)
    return info


def test_plan_matches_oracle_small_dense():
    info = _compare_plan(W.sphere_patches(), p=1, m=2, q=8, gauss_regular=6, dense=True)
    assert info.n_far_blocks == 0
    assert info.n_pairs[1] == 96 and sum(info.n_pairs) == 96 * 97 // 2


def test_plan_matches_oracle_sphere_h2():
    info = _compare_plan(W.sphere_patches(), p=1, m=3, q=4, leaf_depth=1, eta=1.6)
    assert info.n_far_blocks > 0 and info.n_near_blocks > 0


def test_plan_matches_oracle_torus_h2():
    _compare_plan(W.torus_patches(), p=2, m=2, q=4, leaf_depth=1, eta=1.6)


def test_wavenumber_aware_admissibility():
    """kappa_diam > 0 keeps a block out of the far field while kappa max(diam) exceeds it: on the torus at
    kappa = 8 (clusters of patch size span several wavelengths) the partition equals the oracle's under the
    same option, has no far blocks on the coarse levels, and still tiles the block index set (the far
    field moves to finer levels and grows); without the wavenumber (Laplace) the option changes nothing."""
    base = dict(p=1, m=4, q=4, leaf_depth=1, eta=1.6, kernel=1, wavenumber=8.0)
    blind = _compare_plan(W.torus_patches(), **base)
    aware = _compare_plan(W.torus_patches(), kappa_diam=6.0, **base)
    g = igb.Geometry(W.torus_patches())
    _, far_b = igb.Plan(g, mode=igb.IGB_H2_STORED, **base).partition()
    _, far_a = igb.Plan(g, mode=igb.IGB_H2_STORED, kappa_diam=6.0, **base).partition()
    assert far_b[:, 0].min() <= 1 and far_a[:, 0].min() >= 2
    assert aware.n_far_blocks > blind.n_far_blocks and aware.n_near_blocks >= blind.n_near_blocks
    nelem, L = aware.n_elements, aware.leaf_level
    covered = int(np.sum(16 ** (4 - far_a[:, 0].astype(np.int64)))) + aware.n_near_blocks * 16 ** (4 - L)
    assert covered == nelem * nelem
    lap = dict(base, kernel=0, wavenumber=0.0)
    _, far_l = igb.Plan(g, mode=igb.IGB_H2_STORED, **lap).partition()
    _, far_l6 = igb.Plan(g, mode=igb.IGB_H2_STORED, kappa_diam=6.0, **lap).partition()
    assert np.array_equal(far_l, far_l6)


def test_plan_matches_oracle_sphere_p3_m5_q8_full_size():
    """The 6-patch sphere at p=3, 32x32 elements per patch, q=8, eta=1.6: the full workload size."""
    info = _compare_plan(W.sphere_patches(), p=3, m=5, q=8, eta=1.6, gauss_regular=6)
    assert info.n_dof == 7350 and info.n_dof_super == 98304 and info.leaf_level == 4
    assert info.n_pairs[1] == 6144


@pytest.mark.parametrize("mode,q,kernel,flags", [("stored", 8, 0, 1), ("onthefly", 8, 0, 7), ("onthefly", 10, 0, 1),
                                                  ("onthefly", 8, 1, 7), ("onthefly", 10, 1, 7),
                                                  ("onthefly", 11, 1, 1)])
def test_layout_flags(mode, q, kernel, flags):
    """Symmetric near storage always at this size; mirrored far pairs only on the fly, with at most 64
    nodes per cluster for the real kernel and 104 for the complex one; the shared launch of far pairs and
    near blocks wherever the pairs are mirrored (near blocks of up to 256 functions need no LDS)."""
    g = igb.Geometry(W.sphere_patches())
    m = igb.IGB_H2_STORED if mode == "stored" else igb.IGB_H2_ONTHEFLY
    info = igb.Plan(g, p=1, m=4, q=q, eta=1.6, gauss_regular=4, mode=m, kernel=kernel,
                    wavenumber=2.0 if kernel else 0.0).info
    assert info.n_far_blocks > 0
    assert info.layout_flags == flags


def test_single_hip_runtime_in_process():
    """The binding loads torch before libigabem.so, so the library binds to torch's HIP runtime
    instead of bringing a second copy into the process (the second would see no device)."""
    with open("/proc/self/maps") as fh:
        libs = {ln.split()[-1] for ln in fh if "libamdhip64" in ln}
    assert len(libs) == 1, libs


def test_solver_and_network_entry_points_reject_null_arguments():
    """Argument checks that run before any device work."""
    assert igb._lib.igb_solve_fgmres(None, None, None, None, 1e-8, 10, 10, None) == igb.IGB_EINVAL
    assert igb._lib.igb_cnn_training_pairs(None, None, 1, None, None) == igb.IGB_EINVAL
    assert igb._lib.igb_cnn_train_operator(None, None, None, None, 1, 1, 1, 1e-3, None) == igb.IGB_EINVAL
    h = igb.C.c_void_p()
    assert igb._lib.igb_cnn_create(None, 0, None, igb.C.byref(h)) == igb.IGB_EINVAL
    assert igb._lib.igb_cnn_forward(None, None, 1, 1, 1, None) == igb.IGB_EINVAL
    assert igb._lib.igb_cnn_gradient(None, None, None, 1, 1, 1, None, None) == igb.IGB_EINVAL
    assert igb._lib.igb_cnn_train(None, None, None, 1, 1, 1, 1, 1, 1, 1e-3, None) == igb.IGB_EINVAL
    assert igb._lib.igb_cnn_get_weights(None, None) == igb.IGB_EINVAL


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys as _sys
    r = subprocess.run([_sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_plan_matches_oracle_fichera_and_perturbed_sphere():
    """The partition and pair classes on the Fichera cube (re-entrant edges and corner; touching pairs
    across perpendicular faces) and on the perturbed sphere (knots at 1/4 and 3/4) equal the oracle's."""
    info = _compare_plan(W.fichera_patches(), p=1, m=3, q=4, leaf_depth=1, eta=1.6, gauss_regular=6)
    assert info.n_far_blocks > 0 and info.n_pairs[1] == 24 * 64
    assert info.n_pairs[2] > 0 and info.n_pairs[3] > 0
    info = _compare_plan(W.perturbed_mapping_patches(W.sphere_patches()), p=2, m=3, q=4, leaf_depth=1, eta=1.6,
                         gauss_regular=6)
    assert info.n_far_blocks > 0


@pytest.mark.parametrize("gap", [0.85, 0.92])
def test_plan_admissibility_on_two_flat_squares(gap):
    """The product's host plan on two flat unit squares a gap apart (closed-form cluster diameters and
    distances, Sec. 4.2): equal to the oracle's, the squares admissible iff sqrt(2) < 1.6 gap, and
    otherwise every pair of quarters across the gap admissible."""
    a = W.flat_patch([0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0])
    o = 1.0 + gap
    b = W.flat_patch([o, 0, 0], [o + 1, 0, 0], [o, 1, 0], [o + 1, 1, 0])
    _compare_plan([a, b], p=1, m=2, q=4, leaf_depth=1, eta=1.6)
    _, far = igb.Plan(igb.Geometry([a, b]), mode=igb.IGB_H2_STORED, p=1, m=2, q=4, leaf_depth=1,
                      eta=1.6).partition()
    far = {tuple(map(int, r)) for r in far}
    cross1 = {(1, t, s) for t in range(4) for s in range(4, 8)}
    if math.sqrt(2.0) < 1.6 * gap:
        assert (0, 0, 1) in far and not (cross1 & far)
    else:
        assert (0, 0, 1) not in far and cross1 <= far
