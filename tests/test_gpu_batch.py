"""Step graphs, the batched pool and the sort-schedule autotuner (mixed precision).

The current is summed in 64-bit fixed point and every other quantity is
computed per face, edge or particle in a fixed order, so the state after n
steps does not depend on how the launches are issued (eager or replayed
from a graph), on how instances are pooled, or on the sort schedule: all
comparisons here are bit-exact.
"""

import numpy as np
import pytest

import synth
from synth import configs

pytestmark = pytest.mark.gpu

QE, ME = synth.ELECTRON_CHARGE, synth.ELECTRON_MASS


@pytest.fixture(scope="module")
def axp():
    import paper_1701_03784_amd as pkg
    pkg.load_library()
    return pkg


def _state(c):
    E, B = c.get_fields()
    D, J, Q = c.get_sources()
    zr, u, sp = c.get_particles()
    order = np.lexsort((u[:, 2], u[:, 1], u[:, 0], zr[:, 1], zr[:, 0]))
    return dict(E=E, B=B, D=D, J=J, Q=Q, zr=zr[order], u=u[order], sp=sp[order])


def _assert_same(a, b, what):
    for k in a:
        assert a[k].shape == b[k].shape, (what, k)
        assert np.array_equal(a[k], b[k]), (what, k, float(np.abs(a[k] - b[k]).max()))


def _cavity_member(axp, n_part=3000, seed=11, weight=configs.CAVITY_WEIGHT, dt=configs.CAVITY_DT, **kw):
    m = configs.cavity_mesh()
    c = axp.make_ctx(m, dt=dt, **kw)
    E0, B0, _ = synth.tm010_fields(m.nodes, m.tris, c.get_edges(), configs.CAVITY_A, 1e6, c.info()["dt"])
    c.set_fields(E0, B0)
    sp = c.add_species(QE, ME, weight)
    zr, u = configs.cavity_beam(n_part, seed=seed)
    c.inject(sp, zr, u)
    return c


def _tube_member(axp, seed=5, n_part=6000, **kw):
    m = configs.bwo_mesh(seed=seed, h=0.6e-3, n_periods=2, up=0.005, down=0.005)
    c = axp.make_ctx(m, **kw)
    n1, n2 = c.info()["n_edges"], c.info()["n_faces"]
    c.set_fields(np.zeros(n1), np.zeros(n2))
    c.set_external_bz(configs.BWO_BZ)
    L = m.meta["length"]
    sp = c.add_species(QE, ME, configs.bwo_weight(n_part, L))
    zr, u = configs.bwo_beam(n_part, L, seed=seed)
    c.inject(sp, zr, u)
    return c


def test_graph_replays_match_eager(axp):
    print("[gpu] graph vs eager, cavity, 3 x 16 steps", flush=True)
    a = _cavity_member(axp, use_graph=0)
    b = _cavity_member(axp, use_graph=1)
    for rep in range(3):
        a.step(16)
        b.step(16)
        sa, sb = _state(a), _state(b)       # eager work between the replays
        b.diag()
        _assert_same(sa, sb, f"replay {rep}")
    # a step count that is not a multiple of the graph window mixes both paths
    a.step(7)
    b.step(7)
    _assert_same(_state(a), _state(b), "mixed")


def test_batch_matches_members_run_alone(axp):
    print("[gpu] batch of 3 vs alone, 2 x 20 steps", flush=True)

    def members():
        return [_cavity_member(axp), _cavity_member(axp, n_part=2000, seed=12, weight=2 * configs.CAVITY_WEIGHT,
                                                    dt=0.8 * configs.CAVITY_DT),
                _tube_member(axp)]

    alone = members()
    for c in alone:
        c.diag()
        c.step(20)
    ref1 = [_state(c) for c in alone]
    for c in alone:
        c.step(20)
    ref2 = [_state(c) for c in alone]

    pooled = members()
    for c in pooled:
        c.diag()
    b = axp.Batch(pooled)
    info = b.info()
    assert info["n_faces"] == sum(c.info()["n_faces"] for c in pooled)
    b.step(20)
    b.sync()
    for k, c in enumerate(pooled):
        _assert_same(ref1[k], _state(c), f"member {k} after 20")
        assert c.info()["step"] == 20
    b.step(20)
    b.sync()
    for k, c in enumerate(pooled):
        _assert_same(ref2[k], _state(c), f"member {k} after 40")
        d, da = c.diag(), alone[k].diag()
        assert d["n_absorbed"] == da["n_absorbed"]
        assert d["gauss_max_drift"] <= 1e-13 * d["gauss_scale"]
        # the state is the same bit for bit, and so are the evaluations of it
        assert d["W_E_now"] == da["W_E_now"]
        assert d["Q_total"] == da["Q_total"] and d["n_live"] == da["n_live"]
    b.close()


def test_batch_with_diagnostic_steps_matches_members_alone(axp):
    """Members with a diagnostic step every step, pooled (the pool's
    diagnostic steps take the 32-bit charge window of single-charge species):
    the state after 24 steps equals each member stepped alone, with exact
    continuity, and a pool refuses members of different cadences."""
    print("[gpu] batch with diagnostics vs alone", flush=True)

    def members():
        return [_cavity_member(axp, diag_every=1), _cavity_member(axp, n_part=2000, seed=12, diag_every=1),
                _tube_member(axp, diag_every=1)]

    alone = members()
    for c in alone:
        c.step(24)
    ref = [_state(c) for c in alone]
    pooled = members()
    b = axp.Batch(pooled)
    b.step(24)
    b.sync()
    for k, c in enumerate(pooled):
        _assert_same(ref[k], _state(c), f"member {k}")
        d = c.diag()
        assert d["dce_max_abs"] == 0 and d["walk_overflow"] == 0
    b.close()
    with pytest.raises(axp.AxpError):
        axp.Batch([_cavity_member(axp, diag_every=1), _cavity_member(axp, diag_every=2)])


def test_autotune_keeps_results(axp, monkeypatch):
    """Both knobs (sort period, window lead) change where sums land, never
    their values: the tuned run equals a run with the default knobs."""
    print("[gpu] autotune vs fixed schedule", flush=True)
    monkeypatch.delenv("AXP_AUTOTUNE_CACHE", raising=False)
    a = _tube_member(axp, use_graph=1, diag_every=1)
    sp = a.autotune(trial_steps=8)
    info = a.info()
    assert sp in (1, 2, 4, 8, 16) and info["sort_period"] == sp
    assert info["window_lead"] in (64, 128, 192, 256, 320)
    n = info["step"]
    assert n >= 10 * 8                                 # ten trials ran
    b = _tube_member(axp, use_graph=0, diag_every=1)
    assert b.info()["window_lead"] == 192
    b.step(n)
    _assert_same(_state(a), _state(b), "autotuned")
    da, db = a.diag(), b.diag()
    assert da["dce_max_abs"] == db["dce_max_abs"] == 0 and da["Q_total"] == db["Q_total"]


def test_autotune_cache(axp, tmp_path, monkeypatch):
    """A cache hit applies the stored knobs and runs no step; another
    particle count (two powers of two away) is another key."""
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("AXP_AUTOTUNE_CACHE", str(path))
    print("[gpu] autotune cache", flush=True)
    a = _tube_member(axp, use_graph=1)
    sp = a.autotune(trial_steps=4)
    wl = a.info()["window_lead"]
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and lines[0].split()[1:3] == [str(sp), str(wl)]
    assert "gfx950" in lines[0].split()[0]
    b = _tube_member(axp, use_graph=1)
    assert b.autotune(trial_steps=4) == sp
    assert b.info()["window_lead"] == wl and b.info()["step"] == 0
    c = _tube_member(axp, n_part=24000, use_graph=1)
    c.autotune(trial_steps=4)
    assert c.info()["step"] > 0 and len(path.read_text().splitlines()) == 2


def test_batch_rejects_plain_members(axp):
    m = configs.cavity_mesh()
    c = axp.make_ctx(m, precision=axp.PREC_PLAIN_FP64, dt=configs.CAVITY_DT)
    c.add_species(QE, ME, configs.CAVITY_WEIGHT)
    with pytest.raises(axp.AxpError):
        axp.Batch([c])

