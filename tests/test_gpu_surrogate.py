"""The learned screen end to end, on the GPU: solver-labelled designs, training with the
library's BF16 kernels, held-out switching-field error, the gain of a screening round over
random proposals (every pick re-verified by the batched solver, which stays the judge), and a
second round after the judged picks joined the training set."""
import numpy as np
import pytest

from paper_1603_09493_amd import inputs as I

pytestmark = pytest.mark.gpu


def _case(name, **kw):
    print(f"[gpu-case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _progress(msg):
    print(f"[surrogate] {msg}", flush=True)


def test_surrogate_trains_and_screens_better_than_random():
    import torch
    from paper_1603_09493_amd import bpm
    from paper_1603_09493_amd import surrogate as SG
    ctx = bpm.Context(0)
    n_train, n_test, t_end = 896, 128, 0.3e-9
    x = SG.sample(n_train + n_test, seed=12)
    _case("surrogate-label", n=x.shape[0])
    lab = SG.label_designs(ctx, x, t_end=t_end, progress=_progress)
    assert np.all(lab.status == 0)
    frac = lab.switched.mean()
    assert 0.1 < frac < 0.95, frac
    X = SG.scale(x).astype(np.float32)
    tr = slice(0, n_train)
    te = slice(n_train, None)
    lab_tr = SG.Labels(lab.switched[tr], lab.B_sw[tr], lab.t_sw[tr], lab.status[tr], 0, 0)
    lab_te = SG.Labels(lab.switched[te], lab.B_sw[te], lab.t_sw[te], lab.status[te], 0, 0)
    sc = SG.TargetScaler.fit(lab_tr)
    T, mask = sc.targets(lab_tr)
    net = bpm.Mlp(ctx, 512, I.mlp_init_params(3))
    e0, _, _ = SG.bsw_error(net, sc, X[te], lab_te)
    _case("surrogate-train", n=n_train)
    losses = SG.train(net, X[tr], T, mask, epochs=300, batch=64, lr=2e-3)
    assert losses[-1] < 0.4 * losses[0]
    e1, p95, Y = SG.bsw_error(net, sc, X[te], lab_te)
    print(f"[surrogate] held-out |rel err| of B_sw: mean {e1:.4f} p95 {p95:.4f} (untrained {e0:.3f}); "
          f"switched fraction {frac:.2f}", flush=True)
    # the held-out error is data-limited: about 3.3 % at 896 labels, 2.3 % at 1792, 1.75 % at
    # 4864, 1.4 % at 8192 (the bench trains on 8192)
    assert e1 < 0.5 * e0 and e1 < 0.045
    # switching classification on held-out designs
    acc = ((Y[:, 2] > 0) == lab_te.switched).mean()
    assert acc > 0.8, acc
    # screening round: the surrogate's picks against the same number of random stable designs
    _case("surrogate-screen")
    min_stab = 40.0
    picks, secs, scores = SG.screen_round(net, seed=99, n=200_000, k=96, min_stability=min_stab)
    xp = SG.unscale(picks)
    assert np.all(SG.stability(xp) >= min_stab)
    rng = np.random.default_rng(5)
    xr = SG.sample(4000, seed=77)
    xr = xr[SG.stability(xr) >= min_stab][:96]
    assert xr.shape[0] == 96
    lab_p = SG.label_designs(ctx, xp, t_end=t_end, progress=_progress)
    lab_r = SG.label_designs(ctx, xr, t_end=t_end, progress=_progress)
    hit_p, hit_r = lab_p.switched.mean(), lab_r.switched.mean()
    print(f"[surrogate] screen 200k in {secs*1e3:.1f} ms; solver-verified switching: picks {hit_p:.2f} "
          f"vs random {hit_r:.2f}", flush=True)
    assert hit_p >= 0.75 and hit_p >= hit_r + 0.1
    # closing the loop: the judged picks join the training set, training continues, and the next
    # round's picks are judged again
    _case("surrogate-active-round")
    X1 = np.concatenate([X[tr], picks]).astype(np.float32)
    T1p, m1p = sc.targets(lab_p)
    T1 = np.concatenate([T, T1p]).astype(np.float32)
    m1 = np.concatenate([mask, m1p])
    train_n = X1.shape[0]
    X2, T2, m2, lab2, picks2, secs2 = SG.active_round(ctx, net, sc, X1, T1, m1, seed=100, n=200_000, k=64,
                                                       min_stability=min_stab, t_end=t_end, progress=_progress)
    assert X2.shape[0] == train_n + 64 and T2.shape == (train_n + 64, 3)
    hit2 = lab2.switched.mean()
    print(f"[surrogate] round 2 after retraining on {train_n} + 64 designs: solver-verified switching "
          f"{hit2:.2f}", flush=True)
    assert hit2 >= 0.75
    assert np.all(SG.stability(SG.unscale(picks2)) >= min_stab)
    net.close()
    ctx.close()
