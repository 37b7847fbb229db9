"""Batched flow solves: every lattice of a batch ends in the state the single solve gives
it alone (bit-identical velocity fields, equal step counts), whether the check intervals
run as captured graphs or as host launches, with the autotuned or any explicit kernel
variant, and while lattices retire at different checks.  One batch is also held against
the FP64 oracle."""
import sys

import numpy as np
import pytest
import torch

from paper_1410_1921_amd import lbm
from paper_1410_1921_amd import workloads as W

pytestmark = pytest.mark.gpu
E = lbm.LBM_VARIANT_EXPLICIT
NOGRAPH = lbm.LBM_VARIANT_NOGRAPH


def say(*a):
    print("[gpu-batch]", *a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def ragged_batch():
    """Uneven lattices: ragged edges, one-voxel-thin, a slit, and a 64-aligned box."""
    return [dev(W.blob_mask((13, 21, 10), 0.55, 3)), dev(W.blob_mask((1, 12, 12), 0.6, 5)),
            dev(W.slit(5, 11, 3, 9, axis=1)), dev(W.blob_mask((16, 16, 64), 0.5, 8)),
            dev(W.blob_mask((9, 40, 70), 0.45, 11))]


def singles(fluids, **kw):
    return [lbm.lbm_flow_solve(m, want_u=True, **kw) for m in fluids]


def same(batch, ones, us):
    for l, (b, s) in enumerate(zip(batch, ones)):
        assert b["steps"] == s["steps"], l
        assert b["converged"] == s["converged"], l
        assert torch.equal(us[l], s.field), l
        # the sums of a check are reduced in another order than the single solve's
        assert b["k_lattice"] == pytest.approx(s["k_lattice"], rel=1e-12, abs=1e-300), l
        assert b["residual"] == pytest.approx(s["residual"], rel=1e-9), l
        assert np.allclose(b["mean_rho_u"], s["mean_rho_u"], rtol=1e-12, atol=1e-20), l


@pytest.mark.parametrize("collision", [lbm.LBM_COLLIDE_BGK, lbm.LBM_COLLIDE_MRT])
def test_fixed_steps_equal_single_solves(collision):
    fluids = ragged_batch()
    kw = dict(tau=0.7, force=(1e-5, 2e-6, -1e-6), fixed_steps=333, check_every=50,
              collision=collision)
    say("fixed steps, collision", collision)
    st, res, us, sc = lbm.lbm_flow_solve_batch(fluids, want_u=True, **kw)
    assert st == lbm.LBM_OK and sc["group_bytes_run"] in (-1, 128e6, 192e6, 256e6, 384e6)
    same(res, singles(fluids, **kw), us)


@pytest.mark.parametrize("variant", [E, E | lbm.LBM_VARIANT_REMAP, E | lbm.LBM_VARIANT_NTSTORE,
                                     E | lbm.LBM_VARIANT_REMAP | lbm.LBM_VARIANT_NTSTORE])
def test_graph_and_host_launches_agree(variant):
    # fixed runs of 1-4 check intervals: the graph of an interval is replayed up to three
    # times (both parities), each result against the host-launched steps
    fluids = ragged_batch()
    for k in (1, 2, 3, 4):
        kw = dict(tau=0.8, force=(1e-5, 0, 0), fixed_steps=k * 25, check_every=25)
        # two groups (the first four lattices fit 2 MB, the fifth does not)
        _, a, ua, ra = lbm.lbm_flow_solve_batch(fluids, want_u=True, variant=variant,
                                                group_bytes=2_000_000, **kw)
        _, b, ub, rb = lbm.lbm_flow_solve_batch(fluids, want_u=True, variant=variant | NOGRAPH,
                                                group_bytes=2_000_000, **kw)
        assert ra["variant"] == variant and rb["variant"] == variant | NOGRAPH
        assert ra["groups"] == 2
        for l in range(len(fluids)):
            assert torch.equal(ua[l], ub[l]), (k, l)
            assert a[l]["k_lattice"] == b[l]["k_lattice"], (k, l)
        say("variant", variant, "intervals", k, "agree")


def test_retirement_at_different_checks():
    # slits of different widths converge after different numbers of checks; each
    # lattice's steps, convergence and field are those of its own solve
    fluids = [dev(W.slit(4, h + 2, 4, h, axis=1)) for h in (3, 5, 8, 12)] + \
             [dev(W.square_duct(6, 7)), dev(W.slit(3, 4, 11, 9, axis=2))]
    kw = dict(tau=0.9, force=(1e-6, 0, 0), max_steps=200_000, check_every=100, tol=1e-6)
    for variant in (0, NOGRAPH):
        st, res, us, _ = lbm.lbm_flow_solve_batch(fluids, want_u=True, variant=variant, **kw)
        ones = singles(fluids, **kw)
        say("retire steps", [r["steps"] for r in res], [s["steps"] for s in ones])
        assert len({r["steps"] for r in res}) >= 3
        assert st == lbm.LBM_OK and all(r["converged"] for r in res)
        same(res, ones, us)


def test_not_converged_is_reported():
    fluids = [dev(W.slit(4, 14, 4, 12, axis=1)), dev(W.slit(4, 5, 4, 3, axis=1))]
    # tol = 0: a residual of exactly 0 (a binary32 fixed point) does not count either
    st, res, _, _ = lbm.lbm_flow_solve_batch(fluids, tau=0.9, max_steps=400, check_every=100,
                                             tol=0.0)
    assert st == lbm.LBM_W_NOT_CONVERGED
    assert [r["steps"] for r in res] == [400, 400] and not any(r["converged"] for r in res)


def test_batch_against_oracle(orc):
    masks = [W.blob_mask((13, 21, 10), 0.55, 3), W.blob_mask((10, 7, 19), 0.6, 4)]
    kw = dict(tau=0.8, force=(1e-5, 2e-6, 0.0), fixed_steps=400, check_every=100)
    _, res, us, _ = lbm.lbm_flow_solve_batch([dev(m) for m in masks], want_u=True, **kw)
    for l, m in enumerate(masks):
        o = orc.flow_solve(m, **kw)
        u = us[l].cpu().numpy().astype(np.float64)
        assert np.abs(u - o["u"]).max() <= 1e-5 * np.abs(o["u"]).max()
        assert res[l]["k_lattice"] == pytest.approx(o["k_lattice"], rel=1e-4)
        say("oracle k", res[l]["k_lattice"], o["k_lattice"])


def test_reconstructed_batch():
    # a few uneven reconstructions of the batch workload's laws, shrunk to edges 32-64
    fluids = []
    for rp in W.batch_params(6):
        e = rp["n"][0] // 2
        pore, _, _ = lbm.lbm_reconstruct((e, e, e), rp["porosity"], rp["d_mean"] / 2,
                                         rp["d_std"] / 2, rp["d_min"], rp["overlap_tol"],
                                         rp["p_overlap"], rp["seed"])
        fluids.append(pore)
    kw = dict(tau=0.8, force=(1e-6, 0, 0), fixed_steps=300, check_every=100)
    st, res, us, sc = lbm.lbm_flow_solve_batch(fluids, want_u=True, **kw)
    say("reconstructed batch: schedule", sc, "mlups", res[0]["mlups"])
    same(res, singles(fluids, **kw), us)


@pytest.mark.parametrize("group_bytes", [-1, 1, 300_000, 2_000_000])
def test_every_schedule_gives_the_same_state(group_bytes):
    # one group, one lattice per group, and budgets in between, with retirement
    fluids = ragged_batch() + [dev(W.slit(4, 7, 4, 5, axis=1)), dev(W.square_duct(6, 4))]
    kw = dict(tau=0.9, force=(1e-6, 0, 0), max_steps=3000, check_every=100, tol=1e-5)
    st, res, us, sc = lbm.lbm_flow_solve_batch(fluids, want_u=True, group_bytes=group_bytes, **kw)
    ones = singles(fluids, **kw)
    say("schedule", group_bytes, sc["groups"], "groups; steps", [r["steps"] for r in res])
    assert sc["groups"] == {-1: 1, 1: len(fluids)}.get(group_bytes, sc["groups"])
    same(res, ones, us)


# ------------------------------------------------------------------ Knudsen
def kn_batch():
    """Uneven lattices with hashed pore diameters (1-40 voxels) at their fluid voxels."""
    out = []
    for shape, seed in (((19, 10, 14), 2), ((33, 7, 5), 8), ((1, 9, 30), 4), ((16, 16, 64), 6),
                        ((12, 30, 41), 9)):
        m = W.blob_mask(shape, 0.6, seed)
        d = W.hash_field(shape, seed, 1.0, 40.0).astype(np.float64) * m
        out.append((dev(m), dev(d), m, d))
    return out


KN = dict(d_ref_nm=30.0, voxel_nm=1.5, c_in=0.8, c_out=0.3)


def kn_singles(items, c_inits=None, **kw):
    return [lbm.lbm_knudsen_solve(m, d, want_c=True, c_init=None if c_inits is None else c_inits[l],
                                  **KN, **kw) for l, (m, d, _, _) in enumerate(items)]


def kn_same(batch, ones, cs):
    for l, (b, s) in enumerate(zip(batch, ones)):
        assert b["steps"] == s["steps"], l
        assert b["converged"] == s["converged"], l
        assert torch.equal(cs[l], s.field), l
        assert b["Deff_lattice"] == pytest.approx(s["Deff_lattice"], rel=1e-12), l
        assert b["residual"] == pytest.approx(s["residual"], rel=1e-9), l
        assert b["flux_spread"] == pytest.approx(s["flux_spread"], rel=1e-9, abs=1e-15), l
        assert b["tortuosity_local"] == pytest.approx(s["tortuosity_local"], rel=1e-12), l


def test_knudsen_fixed_steps_equal_single_solves():
    items = kn_batch()
    kw = dict(fixed_steps=333, check_every=50)
    st, res, cs, sc = lbm.lbm_knudsen_solve_batch([i[0] for i in items], [i[1] for i in items],
                                                  want_c=True, **KN, **kw)
    assert st == lbm.LBM_OK and sc["group_bytes_run"] in (-1, 128e6, 192e6, 256e6, 384e6)
    kn_same(res, kn_singles(items, **kw), cs)


@pytest.mark.parametrize("variant", [E, E | lbm.LBM_VARIANT_REMAP | lbm.LBM_VARIANT_NTSTORE])
def test_knudsen_graph_and_host_launches_agree(variant):
    items = kn_batch()
    f, d = [i[0] for i in items], [i[1] for i in items]
    for k in (1, 2, 3, 4, 5):
        kw = dict(fixed_steps=k * 25, check_every=25, group_bytes=500_000)
        _, a, ca, sa = lbm.lbm_knudsen_solve_batch(f, d, want_c=True, variant=variant, **KN, **kw)
        _, b, cb, _ = lbm.lbm_knudsen_solve_batch(f, d, want_c=True, variant=variant | NOGRAPH,
                                                  **KN, **kw)
        assert sa["groups"] >= 2
        for l in range(len(items)):
            assert torch.equal(ca[l], cb[l]), (k, l)
            assert a[l]["Deff_lattice"] == b[l]["Deff_lattice"], (k, l)
        say("knudsen variant", variant, "intervals", k, "agree")


def test_knudsen_retirement_and_warm_start():
    # ducts of different lengths converge after different numbers of checks; a warm start
    # (a linear profile) is passed to some lattices only
    items = []
    for nx in (6, 12, 24, 40):
        m = W.square_duct(nx, 3)
        d = np.full(m.shape, 30.0) * m
        items.append((dev(m), dev(d), m, d))
    c0 = [None, dev((np.linspace(0.8, 0.3, 12, dtype=np.float32)[None, None, :] *
                     items[1][2]).astype(np.float32)), None,
          dev((np.float32(0.55) * items[3][2]).astype(np.float32))]
    kw = dict(max_steps=200_000, check_every=100, tol=1e-7)
    f, d = [i[0] for i in items], [i[1] for i in items]
    for variant, gb in ((0, 0), (NOGRAPH, 0), (0, 1), (0, 12000)):
        st, res, cs, _ = lbm.lbm_knudsen_solve_batch(f, d, want_c=True, c_inits=c0,
                                                     variant=variant, group_bytes=gb, **KN, **kw)
        ones = kn_singles(items, c_inits=c0, **kw)
        say("knudsen retire steps", [r["steps"] for r in res], [s["steps"] for s in ones])
        assert len({r["steps"] for r in res}) >= 3
        assert st == lbm.LBM_OK and all(r["converged"] for r in res)
        kn_same(res, ones, cs)


def test_knudsen_batch_against_oracle(orc):
    items = kn_batch()[:3]
    kw = dict(fixed_steps=400, check_every=50)
    _, res, cs, _ = lbm.lbm_knudsen_solve_batch([i[0] for i in items], [i[1] for i in items],
                                                want_c=True, **KN, **kw)
    for l, (_, _, m, d) in enumerate(items):
        tg = np.where(m == 1, orc.tau_g(d, 20.0, 1.0), 1.0)
        o = orc.knudsen_solve(m, tg, 0.8, 0.3, **kw)
        assert np.abs(cs[l].cpu().numpy() - o["c"]).max() < 1e-5
        assert res[l]["Deff_lattice"] == pytest.approx(o["Deff_lattice"], rel=1e-4)
        say("knudsen oracle", res[l]["Deff_lattice"], o["Deff_lattice"])
