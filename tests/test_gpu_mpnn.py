"""GPU parity of the learned smooth-vector network (amg_mpnn_*).

Against the numpy oracle (oracle/mpnn.py, its backward pass pinned by finite
differences on the CPU), with the oracle emulating the bfloat16 storage:
  * features: equal up to one bfloat16 unit in the last place;
  * forward prediction y: relative L2 error <= 2e-2;
  * gradient of the loss: relative L2 error <= 5e-2 per parameter block,
    loss within 2e-2 relative;
and the properties the method needs: training lowers the loss, and the
predicted vector is positive, finite and drives a working hierarchy.  At the
learned form's full size (the 128^3 log-normal field, seeded weights) the
prediction is compared with the oracle's stored one
(tests/golden/oracle_learned128.json): sampled entries within 2e-2 of the
vector's RMS, its norm within 2e-2 relative.
The prediction itself is "parity unpinned" beyond this (trained weights have
no closed form); bench.py measures it by PCG iterations.
"""
import json
import os

import numpy as np
import pytest

import oracle
import oracle.mpnn as M
import workloads as W

from gpu_helpers import dev, host, require_gpu, say, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _net(theta=None):
    import paper_2303_02352_amd as amd
    return amd.SmoothVectorNet(theta)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, float) - np.asarray(b, float)) / max(1e-30, np.linalg.norm(b)))


@pytest.mark.parametrize("N,seed", [(12, 3), (17, 5)])
def test_features_match_oracle(N, seed):
    A = W.lognormal7(N, seed, ell=4.0)
    say("mpnn features", N, seed)
    Xg = _net().features(dev(A.row_ptr), dev(A.col), dev(A.val))
    Xo = M.round_bf16(M.features(A)[0])
    ulp = np.maximum(np.abs(Xo), 1e-30) * 2.0 ** -7
    assert np.all(np.abs(Xg - Xo) <= ulp + 1e-12), np.max(np.abs(Xg - Xo) / ulp)


@pytest.mark.parametrize("N,seed", [(12, 3), (21, 8)])
def test_forward_matches_oracle(N, seed):
    A = W.lognormal7(N, seed, ell=4.0)
    theta = M.init_params(seed).astype(np.float32)
    say("mpnn forward", N, seed)
    yg = _net(theta).predict(dev(A.row_ptr), dev(A.col), dev(A.val), want_y=True)
    yo, _ = M.forward(theta.astype(np.float64), A, bf16=True)
    err = _rel(yg, yo)
    say("  rel L2 %.2e" % err)
    assert err <= 2e-2


def test_forward_full_size_against_stored_oracle():
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_learned128.json")))
    A = W.lognormal7(g["n_edge"], g["field_seed"])
    theta = M.init_params(g["theta_seed"]).astype(np.float32)
    say("mpnn forward full size", A.n)
    w = torch.empty(A.n, dtype=torch.float64, device="cuda")
    yg = _net(theta).predict(dev(A.row_ptr), dev(A.col), dev(A.val), w_out=w, want_y=True)
    rows = np.asarray(g["rows"], dtype=np.int64)
    ref = np.array([float.fromhex(h) for h in g["y"]])
    rms = g["norm_y"] / np.sqrt(A.n)
    err = float(np.max(np.abs(yg[rows].astype(np.float64) - ref))) / rms
    nrm = float(np.linalg.norm(yg.astype(np.float64)))
    say("  sampled max err / rms %.2e, norm %.6g vs %.6g" % (err, nrm, g["norm_y"]))
    assert err <= 2e-2
    assert abs(nrm - g["norm_y"]) <= 2e-2 * g["norm_y"]
    wh = host(w)
    assert np.all(np.isfinite(wh)) and np.all(wh > 0)


def test_gradient_matches_oracle():
    A = W.lognormal7(14, 4, ell=4.0)
    theta = M.init_params(7).astype(np.float32)
    target = 0.2 + W.uniform(60, A.n)
    say("mpnn gradient")
    loss_g, g = _net(theta).train_step(dev(A.row_ptr), dev(A.col), dev(A.val), dev(target), 0.0,
                                       want_grad=True)
    loss_o, go = M.loss_and_grad(theta.astype(np.float64), A, np.log(target), bf16=True)
    say("  loss gpu %.6e oracle %.6e" % (loss_g, loss_o))
    assert abs(loss_g - loss_o) <= 2e-2 * loss_o
    o = 0
    for name, shp in M.SHAPES:
        m = int(np.prod(shp))
        err = _rel(g[o:o + m], go[o:o + m])
        say("  %s rel L2 %.2e" % (name, err))
        assert err <= 5e-2, name
        o += m


def test_training_lowers_loss_and_vector_drives_hierarchy():
    import paper_2303_02352_amd as amd
    from paper_2303_02352_amd import surrogate
    fields = [W.lognormal7(16, s, ell=4.0) for s in (30, 31)]
    data = []
    for A in fields:
        csr = surrogate.device_csr(A, torch)
        data.append(csr + (surrogate.relax_target(csr, torch),))
    net = _net(surrogate.init_params(1))
    hist = surrogate.train(net, data, 120, 3e-3, log_every=0)
    say("  loss %.3e -> %.3e" % (hist[0], hist[-1]))
    assert np.mean(hist[-10:]) < 0.5 * np.mean(hist[:10])
    A = W.lognormal7(16, 32, ell=4.0)
    csr = surrogate.device_csr(A, torch)
    w = torch.empty(A.n, dtype=torch.float64, device="cuda")
    net.predict(*csr, w_out=w)
    assert bool(torch.isfinite(w).all()) and bool((w > 0).all())
    H = amd.Hierarchy(*csr, model_params=net.params())
    assert H.info()["smooth_status"] == amd.AMG_OK
    xs, b = W.manufactured_rhs(A, 1)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    st, it, rel = H.solve(dev(b), x)
    assert st == 0 and rel <= 1e-6
    # the learned vector goes through the same setup as any other: oracle parity
    Ho = oracle.Hierarchy(A, oracle.AMGParams(smooth_vec=2), w=host(w))
    assert H.info()["n"] == [s[0] for s in Ho.sizes()]


def _levels_equal(H1, H2):
    assert H1.info()["n"] == H2.info()["n"]
    for k in range(H1.info()["levels"]):
        a, b = H1.export_level(k), H2.export_level(k)
        for f in ("row_ptr", "col", "agg"):
            assert (a[f] is None and b[f] is None) or np.array_equal(a[f], b[f]), (k, f)
        for f in ("val", "w", "pval", "dinv"):
            if a[f] is not None:
                assert np.array_equal(a[f].view(np.uint64), b[f].view(np.uint64)), (k, f)


def test_learned_mode_through_the_c_abi():
    """AMG_SMOOTH_LEARNED in amg_setup: the same hierarchy as AMG_SMOOTH_GIVEN
    with the network's prediction, and smooth_status OK."""
    import paper_2303_02352_amd as amd
    from paper_2303_02352_amd import surrogate
    A = W.lognormal7(24, 7, ell=4.0)
    rp, ci, va = dev(A.row_ptr), dev(A.col), dev(A.val)
    params, meta = surrogate.load_params()
    net = amd.SmoothVectorNet(params)
    w = torch.empty(A.n, dtype=torch.float64, device="cuda")
    net.predict(rp, ci, va, w_out=w)
    Hg = amd.Hierarchy(rp, ci, va, smooth_vector=w)
    Hl = amd.Hierarchy(rp, ci, va, model_params=params)
    assert Hl.info()["smooth_status"] == amd.AMG_OK
    _levels_equal(Hl, Hg)


def test_learned_setups_reuse_the_network_across_sizes_and_parameters():
    """The setup keeps one network per device: learned setups of growing and
    shrinking sizes, with two parameter sets, each equal to the GIVEN path
    with a fresh network's prediction."""
    import paper_2303_02352_amd as amd
    from paper_2303_02352_amd import surrogate
    p1, _ = surrogate.load_params()
    p2 = M.init_params(11).astype(np.float32)
    for N, params in ((12, p1), (30, p2), (9, p1), (30, p1)):
        A = W.lognormal7(N, 40 + N, ell=4.0)
        rp, ci, va = dev(A.row_ptr), dev(A.col), dev(A.val)
        w = torch.empty(A.n, dtype=torch.float64, device="cuda")
        amd.SmoothVectorNet(params).predict(rp, ci, va, w_out=w)
        say("learned setup n=%d" % A.n)
        Hl = amd.Hierarchy(rp, ci, va, model_params=params)
        assert Hl.info()["smooth_status"] == amd.AMG_OK
        _levels_equal(Hl, amd.Hierarchy(rp, ci, va, smooth_vector=w))


def test_learned_mode_from_a_model_file(tmp_path):
    """model_path instead of model_params: the same hierarchy; a file that
    cannot be read falls back to relaxation with smooth_status MODEL."""
    import paper_2303_02352_amd as amd
    from paper_2303_02352_amd import surrogate
    A = W.lognormal7(20, 9, ell=4.0)
    rp, ci, va = dev(A.row_ptr), dev(A.col), dev(A.val)
    params, meta = surrogate.load_params()
    Hp = amd.Hierarchy(rp, ci, va, model_params=params)
    Hf = amd.Hierarchy(rp, ci, va, model_path=surrogate.DEFAULT_MODEL)
    assert Hf.info()["smooth_status"] == amd.AMG_OK
    _levels_equal(Hf, Hp)
    Hm = amd.Hierarchy(rp, ci, va, model_path=tmp_path / "missing.json", smooth_sweeps=20)
    Hr = amd.Hierarchy(rp, ci, va, smooth_vec=amd.AMG_SMOOTH_RELAX, smooth_sweeps=20)
    assert Hm.info()["smooth_status"] == amd.AMG_ERR_MODEL
    _levels_equal(Hm, Hr)


@pytest.mark.parametrize("bias", [1e30, -1e30])
def test_learned_mode_falls_back_to_relaxation(bias):
    """A parameter set whose prediction overflows (w = inf) or underflows
    (w = 0): amg_setup succeeds with the relaxation vector and reports
    AMG_ERR_MODEL in smooth_status; the hierarchy is the RELAX one bit for bit."""
    import paper_2303_02352_amd as amd
    A = W.lognormal7(16, 5, ell=4.0)
    rp, ci, va = dev(A.row_ptr), dev(A.col), dev(A.val)
    theta = np.zeros(amd.AMG_MPNN_NPARAMS, np.float32)
    theta[-1] = bias
    Hl = amd.Hierarchy(rp, ci, va, model_params=theta, smooth_sweeps=20)
    Hr = amd.Hierarchy(rp, ci, va, smooth_vec=amd.AMG_SMOOTH_RELAX, smooth_sweeps=20)
    inf = Hl.info()
    say("fallback bias %g: smooth_status %d" % (bias, inf["smooth_status"]))
    assert inf["smooth_status"] == amd.AMG_ERR_MODEL
    _levels_equal(Hl, Hr)
