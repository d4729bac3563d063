"""Learned SPAI on the GPU: the network's kernels against the FP64 oracle,
the pair features against the oracle's, training, and what the trained
network gains.

Bounds: forward within FP32 rounding (1e-5 of the output scale); the loss
to 1e-5 relative and the gradient to 1e-4 of its largest entry (FP32 sums
over ~1,000 samples); Adam to 1e-6 (FP32 moments); features to 1e-5
(FP32 storage of FP64 values, summation order of the matrix powers).
"""

import time

import numpy as np
import pytest

import synth
from synth import configs
from oracle import mlp as om
from oracle.hodge import hodge_eps
from oracle.spai import spai
from oracle.topology import build_topology

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def axp():
    import paper_1701_03784_amd as pkg
    pkg.load_library()
    return pkg


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("H,L", [(64, 2), (32, 1), (64, 3)])
def test_mlp_forward_and_gradient_match_oracle(axp, torch, H, L):
    print(f"[gpu] mlp H={H} L={L}", flush=True)
    rng = np.random.default_rng(H + L)
    net = axp.Mlp(n_hidden=H, n_layers=L, seed=1)
    p = rng.normal(0, 0.3, net.n_params()).astype(np.float32)
    net.set_params(p)
    n = 1037                          # ragged against the 256-sample blocks and 512-sample chunks
    X = rng.normal(size=(n, 16)).astype(np.float32)
    y = rng.normal(size=n).astype(np.float32)
    w = rng.uniform(0.5, 2.0, n).astype(np.float32)
    Xd, yd, wd = _dev(torch, X), _dev(torch, y), _dev(torch, w)
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    net.forward(Xd, out)
    torch.cuda.synchronize()
    po, _ = om.forward(p.astype(np.float64), X, 16, H, L)
    assert np.abs(out.cpu().numpy() - po).max() <= 1e-5 * np.abs(po).max() + 1e-6
    loss, g = net.loss_grad(Xd, yd, wd, want_grad=True)
    lo, go = om.loss_grad(p.astype(np.float64), X, y, w, 16, H, L)
    assert loss == pytest.approx(lo, rel=1e-5)
    assert np.abs(g - go).max() <= 1e-4 * np.abs(go).max()


def test_mlp_adam_matches_oracle(axp, torch):
    rng = np.random.default_rng(5)
    net = axp.Mlp(n_hidden=64, n_layers=2, seed=3)
    p = net.get_params().astype(np.float64)
    n = 700
    X = rng.normal(size=(n, 16))
    y = rng.normal(size=n)
    Xd, yd, wd = _dev(torch, X), _dev(torch, y), _dev(torch, np.ones(n))
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t in range(1, 4):
        _, g = net.loss_grad(Xd, yd, wd, want_grad=True)
        net.adam_step(1e-3)
        p, m, v = om.adam(p, g.astype(np.float64), m, v, t, 1e-3)
    assert np.abs(net.get_params() - p).max() <= 1e-6
    assert net.info()["adam_steps"] == 3


def test_mlp_save_load(axp, tmp_path):
    net = axp.Mlp(n_hidden=32, n_layers=2, seed=7)
    path = tmp_path / "net.bin"
    net.save(path)
    other = axp.Mlp.load(path)
    assert np.array_equal(other.get_params(), net.get_params())
    assert other.info()["n_hidden"] == 32 and other.info()["spai_level"] == 3


def _oracle_setup(m):
    topo = build_topology(m.nodes, m.tris, m.seg, m.tag)
    assert np.array_equal(topo.edges, synth.canonical_edges(m.tris))
    return topo, hodge_eps(topo)


def test_pair_features_and_targets_match_oracle(axp):
    m = configs.cavity_mesh()
    c = axp.make_ctx(m, dt=configs.CAVITY_DT)
    X, y, kj = c.spai_pairs()
    topo, A = _oracle_setup(m)
    k, j, Xo = om.pair_features(topo, A, 3)
    o1 = np.lexsort((kj[:, 1], kj[:, 0]))
    o2 = np.lexsort((j, k))
    assert np.array_equal(kj[o1, 0], k[o2]) and np.array_equal(kj[o1, 1], j[o2])
    assert np.allclose(X[o1], Xo[o2], rtol=1e-5, atol=1e-6)
    Mo = spai(A, topo.edge_free, 3, 1e-3)
    yo = om.scaled_targets(Mo, A, topo.edge_free, k[o2], j[o2])
    assert np.abs(y[o1] - yo).max() <= 1e-6 * np.abs(yo).max()


def _tube(seed, h, amp, period, taper=0.0):
    return configs.bwo_mesh(seed=seed, h=h, amp=amp, period=period, n_periods=2, up=0.004, down=0.004, taper=taper)


@pytest.fixture(scope="module")
def trained(axp):
    from paper_1701_03784_amd.learned_spai import training_pairs, train
    meshes = [_tube(300 + i, 0.5e-3, 0.001 + 0.0007 * i, 0.012 + 0.002 * i, 0.1 * i) for i in range(4)]
    X, y = training_pairs(meshes, log=lambda s: print("[gpu]", s, flush=True))
    net = axp.Mlp(n_hidden=64, n_layers=2, seed=0)
    t0 = time.perf_counter()
    hist = train(net, X, y, epochs=60, batch=4096, lr=3e-3, lr_final=1e-4,
                 log=lambda s: print("[gpu]", s, flush=True) if s.endswith("9") or s.startswith("epoch 0") else None)
    print(f"[gpu] trained on {len(y)} pairs in {time.perf_counter() - t0:.1f} s", flush=True)
    return net, hist


def test_training_reduces_the_loss(trained):
    net, hist = trained
    assert hist[-1] < hist[0] / 5


def test_learned_spai_gain_fallback_and_guard(axp, torch, trained):
    net, _ = trained
    m = _tube(950, 0.45e-3, 0.0021, 0.015, 0.2)            # not among the training meshes
    cp = axp.make_ctx(m)
    X, y, kj = cp.spai_pairs()
    Xd = _dev(torch, X)
    out = torch.empty(len(y), dtype=torch.float32, device="cuda")
    net.forward(Xd, out)
    pred = out.cpu().numpy()
    topo, A = _oracle_setup(m)
    idx, Ah, s = om.scaled_free_hodge(A, topo.edge_free)
    pos = np.full(topo.edges.shape[0], -1)
    pos[idx] = np.arange(len(idx))
    kk, jj = pos[kj[:, 0]], pos[kj[:, 1]]
    jac = (kk == jj).astype(float)
    rl = [om.cgnr_refine(Ah, kk, jj, pred, q)[1] for q in range(4)]
    rj = [om.cgnr_refine(Ah, kk, jj, jac, q)[1] for q in range(4)]
    rp = om.cgnr_refine(Ah, kk, jj, y, 0)[1]                 # the plain SPAI's columns (dropped, symmetrised)
    print("[gpu] mean column residual by CGNR steps: learned start", [f"{r.mean():.4f}" for r in rl],
          "Jacobi start", [f"{r.mean():.4f}" for r in rj], f"plain SPAI {rp.mean():.4f}", flush=True)
    # the gain: the network starts CGNR where the Jacobi guess needs several steps to get
    assert rl[0].mean() < rj[0].mean() / 5
    assert rl[3].mean() < rj[3].mean() / 2
    assert rl[3].mean() < 2.5 * rp.mean()
    # the library's construction: the same refinement, per-column fallback, energy guard
    row_tol = 0.02
    cl = axp.make_ctx(m, spai_model=net, spai_row_tol=row_tol, spai_iters=3)
    il, ip = cl.info(), cp.info()
    assert il["spai_mode"] == axp.SPAI_LEARNED
    kept = rl[3] <= row_tol
    assert il["spai_fallback_columns"] == int((~kept).sum())
    assert il["spai_fallback_columns"] < 0.1 * len(idx)
    assert il["spai_kept_resid_mean"] == pytest.approx(rl[3][kept].mean(), rel=1e-6)
    assert il["spai_pred_resid_mean"] == pytest.approx(rl[0].mean(), rel=1e-6)
    assert il["spai_energy_drift"] <= 1e-6
    print(f"[gpu] SPAI setup: learned {il['spai_seconds']:.3f} s ({il['spai_fallback_columns']} fallback columns), "
          f"plain {ip['spai_seconds']:.3f} s; fro residual learned {il['spai_fro_residual']:.4f} "
          f"plain {ip['spai_fro_residual']:.4f}; dt_cfl learned {il['dt_cfl']:.4e} plain {ip['dt_cfl']:.4e}", flush=True)
    assert il["dt_cfl"] == pytest.approx(ip["dt_cfl"], rel=0.05)
    # a PIC run with the learned M keeps the continuity equation and Gauss's law
    L = m.meta["length"]
    zr, u = configs.bwo_beam(4000, L, seed=4)
    res = {}
    for name, c in (("learned", cl), ("plain", cp)):
        c.set_fields(np.zeros(c.info()["n_edges"]), np.zeros(c.info()["n_faces"]))
        c.set_external_bz(1.0)
        sp_ = c.add_species(synth.ELECTRON_CHARGE, synth.ELECTRON_MASS, configs.bwo_weight(4000, L))
        c.inject(sp_, zr, u)
        c.diag()
        c.step(100)
        d = c.diag()
        assert d["dce_max_abs"] == 0
        assert d["gauss_max_drift"] <= 1e-13 * d["gauss_scale"]
        res[name] = c.get_fields()[0]
    diff = np.linalg.norm(res["learned"] - res["plain"]) / np.linalg.norm(res["plain"])
    print(f"[gpu] E after 100 beam steps, learned vs plain SPAI: rel-L2 {diff:.2e}", flush=True)
    assert diff < 0.05


def test_guard_rejects_a_broken_network(axp):
    # a network that predicts a large constant gives an indefinite M: every
    # column fails the residual test and is rebuilt by least squares, so the
    # result equals the plain SPAI
    net = axp.Mlp(n_hidden=32, n_layers=1, seed=0)
    p = np.zeros(net.n_params(), dtype=np.float32)
    p[-1] = 5.0                                    # output bias
    net.set_params(p)
    m = configs.cavity_mesh()
    cl = axp.make_ctx(m, dt=configs.CAVITY_DT, spai_model=net, spai_row_tol=0.02)
    cp = axp.make_ctx(m, dt=configs.CAVITY_DT)
    assert cl.info()["spai_fallback_columns"] == cl.info()["n_free_edges"]
    Ml, Mp = cl.get_spai(), cp.get_spai()
    assert abs(Ml - Mp).max() <= 1e-12 * abs(Mp).max()


def test_shipped_network_on_the_bwo_profile(axp):
    # the network trained by train_spai.py (seeded tubes, seeds 1000-1255) on a
    # tube it was not trained on: the construction keeps most of its columns
    net = axp.default_spai_model()
    assert net.info()["spai_level"] == 3
    m = _tube(777, 0.35e-3, 0.0025, 0.0167)
    cl = axp.make_ctx(m, spai_model=net, spai_row_tol=0.02, spai_iters=3)
    cp = axp.make_ctx(m)
    il, ip = cl.info(), cp.info()
    print(f"[gpu] shipped network: {il['spai_fallback_columns']} of {il['n_free_edges']} columns fell back; "
          f"start residual {il['spai_pred_resid_mean']:.4f}, refined {il['spai_kept_resid_mean']:.4f}; "
          f"fro learned {il['spai_fro_residual']:.4f} plain {ip['spai_fro_residual']:.4f}", flush=True)
    assert il["spai_mode"] == axp.SPAI_LEARNED
    assert il["spai_fallback_columns"] < 0.05 * il["n_free_edges"]
    assert il["spai_pred_resid_mean"] < 0.03
    assert il["spai_fro_residual"] < 1.5 * ip["spai_fro_residual"]


def test_native_trainer_and_model_file(axp, torch, tmp_path):
    """axp_spai_model_train (through the C ABI) on two tubes written with
    write_mesh, then axp_spai_model_load into a context on an unseen tube.
    The saved network is 16 -> 64 -> 64 -> 1 at level 3 (the file holds
    the sizes and parameters, not the Adam state).  Its loss on the training
    pairs is below a fifth of the same seed's untrained network.  The SPAI
    built from the file is the learned one, accepted by the energy guard,
    with under 10 % of the columns falling back to least squares."""
    meshes = [_tube(310 + i, 0.5e-3, 0.0012 + 0.0008 * i, 0.013 + 0.002 * i) for i in range(2)]
    paths = []
    for i, m in enumerate(meshes):
        p = tmp_path / f"tube{i}.mesh"
        axp.write_mesh(p, m)
        paths.append(str(p))
    lst = tmp_path / "meshes.txt"
    lst.write_text("# training tubes\n" + "\n".join(paths) + "\n\n")
    out = tmp_path / "spai_model.bin"
    Xs, ys = [], []
    for m in meshes:
        c = axp.make_ctx(m, spai_level=3, dt=1e-30)
        X, y, _ = c.spai_pairs()
        c.close()
        Xs.append(X)
        ys.append(y)
    n_pairs = sum(min(150000, len(y)) for y in ys)
    print(f"[gpu] native trainer: {n_pairs} pairs", flush=True)
    axp.spai_model_train(lst, out, seed=7)
    net = axp.Mlp.load(str(out))
    info = net.info()
    assert (info["n_in"], info["n_hidden"], info["n_layers"], info["spai_level"]) == (16, 64, 2, 3)
    X = torch.from_numpy(np.concatenate(Xs).astype(np.float32)).cuda()
    y = torch.from_numpy(np.concatenate(ys).astype(np.float32)).cuda()
    w = torch.ones(len(y), dtype=torch.float32, device="cuda")
    fresh = axp.Mlp(n_hidden=64, n_layers=2, seed=7)
    l_trained, l_fresh = net.loss_grad(X, y, w), fresh.loss_grad(X, y, w)
    print(f"[gpu] native trainer: loss {l_fresh:.3e} untrained -> {l_trained:.3e}", flush=True)
    assert l_trained < l_fresh / 5
    m3 = _tube(320, 0.5e-3, 0.0015, 0.014)
    c = axp.Ctx()
    c.set_mesh(m3.nodes, m3.tris)
    c.set_boundary(m3.seg, m3.tag)
    c.spai_model_load(str(out))
    c.build()
    il = c.info()
    assert il["spai_mode"] == axp.SPAI_LEARNED
    assert il["spai_energy_drift"] <= 1e-6
    assert il["spai_fallback_columns"] < 0.1 * il["n_edges"]
    with pytest.raises(axp.AxpError):
        c.spai_model_load(str(out))                      # after axp_build
    c.close()
    c2 = axp.Ctx()
    with pytest.raises(axp.AxpError):
        c2.spai_model_load(str(tmp_path / "missing.bin"))
    c2.close()
    with pytest.raises(axp.AxpError):
        axp.spai_model_train(tmp_path / "missing.txt", out, seed=7)
    bad = tmp_path / "bad.txt"
    bad.write_text(str(tmp_path / "meshes.txt") + "\n")   # a list file is not a mesh file
    with pytest.raises(axp.AxpError):
        axp.spai_model_train(bad, out, seed=7)
