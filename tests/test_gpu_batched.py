"""Batched epochs of uneven size against a shared reference (persistent work-queue launch,
graph-captured optimiser steps, autotuned tile shape), checked epoch by epoch against the
FP64 oracle on the same crops.  Same bars as the single-pair tests: gradient 1e-5,
fitted K / P / B0 1e-4."""
import numpy as np
import pytest
import torch

import oracle
from synthetic import starfield as sf

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def dia():
    import paper_2104_13715_amd as d
    return d


def gpu(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


@pytest.fixture(scope="module")
def small_batch():
    # 7 epochs of side 120..400 cut from a 512^2 shared reference, 17x17 kernels (the uneven-batch recipe)
    return sf.batched(40, 7, 17, 512, 1900, (120, 400))


def crop_R(batch, e):
    ep = batch.epochs[e]
    s0, s1 = ep.I.shape
    return batch.R[ep.row0:ep.row0 + s0, ep.col0:ep.col0 + s1]


def epochs_gpu(dia, batch):
    return [dia.Epoch(I=gpu(e.I), ref_row0=e.row0, ref_col0=e.col0) for e in batch.epochs]


def objs(dia, batch, rho="gauss"):
    o = dia.Objective(rho=rho, var="ccd_data", sigma0=batch.sigma0_adu, gain=batch.gain, c=2.3849)
    oo = oracle.Objective(rho=rho, var="ccd_data", sigma0=batch.sigma0_adu, gain=batch.gain, c=2.3849)
    return o, oo


@pytest.mark.parametrize("rho", ["gauss", "cauchy"])
def test_loss_grad_batched_matches_oracle_per_epoch(dia, small_batch, rho):
    b = small_batch
    m = b.m
    o, oo = objs(dia, b, rho)
    rng = np.random.default_rng(4)
    th = np.stack([np.concatenate([e.K_true.ravel(), [e.B0_true]]) * rng.uniform(0.9, 1.1, m * m + 1)
                   for e in b.epochs]).astype(np.float32)
    loss, grad = dia.loss_grad_batched(gpu(b.R), epochs_gpu(dia, b), gpu(th), m, o)
    loss, grad = loss.cpu().numpy(), grad.cpu().double().numpy()
    for k, e in enumerate(b.epochs):
        L_ref, g_ref = oracle.loss_grad(crop_R(b, k), e.I, th[k], m, oo)
        eK = np.linalg.norm(grad[k, :-1] - g_ref[:-1]) / np.linalg.norm(g_ref[:-1])
        eB = abs(grad[k, -1] - g_ref[-1]) / abs(g_ref[-1])
        assert eK <= 1e-5 and eB <= 1e-5, (k, eK, eB)
        assert abs(loss[k] - L_ref) <= 2e-6 * abs(L_ref), (k, loss[k], L_ref)


def test_loss_grad_batched_equals_single_pair_path(dia, small_batch):
    b = small_batch
    m = b.m
    o, _ = objs(dia, b)
    th = np.stack([oracle.init_theta(e.I, m) for e in b.epochs]).astype(np.float32)
    Rg = gpu(b.R)
    loss, grad = dia.loss_grad_batched(Rg, epochs_gpu(dia, b), gpu(th), m, o)
    for k, e in enumerate(b.epochs):
        s0, s1 = e.I.shape
        L1, g1 = dia.loss_grad(Rg[e.row0:e.row0 + s0, e.col0:e.col0 + s1], gpu(e.I), gpu(th[k]), m, o)
        g1 = g1.cpu().double().numpy()
        gb = grad[k].cpu().double().numpy()
        assert np.linalg.norm(gb - g1) <= 1e-6 * np.linalg.norm(g1)
        assert abs(loss[k].item() - L1.item()) <= 1e-9 * abs(L1.item())


def test_fit_batched_matches_oracle_per_epoch(dia, small_batch):
    b = small_batch
    m = b.m
    o, oo = objs(dia, b)
    theta, res, st = dia.fit_batched(gpu(b.R), epochs_gpu(dia, b), m, o)
    assert st >= 0
    th = theta.cpu().double().numpy()
    for k, e in enumerate(b.epochs):
        ref = oracle.solve(crop_R(b, k), e.I, m, oo)
        K, Kr = th[k, :-1], ref[:-1]
        eK = np.linalg.norm(K - Kr) / np.linalg.norm(Kr)
        eP = abs(K.sum() - Kr.sum()) / abs(Kr.sum())
        eB = abs(th[k, -1] - ref[-1]) / max(abs(ref[-1]), 1.0)
        print(f"epoch {k} side {e.I.shape[0]}: K {eK:.2e} P {eP:.2e} B0 {eB:.2e} evals {res[k].n_eval} "
              f"stop {res[k].stop}")
        assert res[k].status >= 0
        assert eK <= 1e-4 and eP <= 1e-4 and eB <= 1e-4


def test_loss_grad_batched_pinned_tile_shapes_agree(dia, small_batch, monkeypatch):
    b = small_batch
    m = b.m
    o, _ = objs(dia, b)
    th = np.stack([oracle.init_theta(e.I, m) for e in b.epochs]).astype(np.float32)
    grads = []
    for v in ("1", "2", "3", "4"):  # the narrow shape (5) is a single-pair shape
        monkeypatch.setenv("DIA_TILE_VARIANT", v)
        _, g = dia.loss_grad_batched(gpu(b.R), epochs_gpu(dia, b), gpu(th), m, o)
        grads.append(g.cpu().double().numpy())
    for g in grads[1:]:
        assert np.linalg.norm(g - grads[0]) <= 1e-6 * np.linalg.norm(grads[0])


def test_fit_batched_rejects_bad_epochs(dia, small_batch):
    b = small_batch
    o, _ = objs(dia, b)
    e = b.epochs[0]
    bad = [dia.Epoch(I=gpu(e.I), ref_row0=b.R.shape[0] - 10, ref_col0=0)]
    with pytest.raises(dia.DIAError) as ex:
        dia.fit_batched(gpu(b.R), bad, b.m, o)
    assert ex.value.status == dia.E_SIZE


def test_loss_grad_batched_uneven_full_size_sampled(dia):
    # the 64-epoch uneven batch (sides 512..2048 against a shared 2048^2 reference, m = 17) in one
    # persistent launch; the smallest and the largest epochs are checked against the oracle
    b = sf.config4()
    m = b.m
    o, oo = objs(dia, b)
    th = np.stack([np.r_[e.K_true.ravel() * 0.97, e.B0_true + 1.0] for e in b.epochs]).astype(np.float32)
    loss, grad = dia.loss_grad_batched(gpu(b.R), epochs_gpu(dia, b), gpu(th), m, o)
    torch.cuda.synchronize()
    sides = [e.I.shape[0] for e in b.epochs]
    for k in (int(np.argmin(sides)), int(np.argmax(sides))):
        L_ref, g_ref = oracle.loss_grad(crop_R(b, k), b.epochs[k].I, th[k], m, oo)
        g = grad[k].cpu().double().numpy()
        eK = np.linalg.norm(g[:-1] - g_ref[:-1]) / np.linalg.norm(g_ref[:-1])
        eB = abs(g[-1] - g_ref[-1]) / abs(g_ref[-1])
        print(f"epoch {k} side {sides[k]}: grad rel err dK {eK:.2e} dB0 {eB:.2e}")
        assert eK <= 1e-5 and eB <= 1e-5
        assert abs(loss[k].item() - L_ref) <= 2e-6 * abs(L_ref)


def _golden(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "batched_oracle_thetas.npz")
    if not os.path.exists(path):
        pytest.skip("batched_oracle_thetas.npz not written (tests/golden/make_batched_oracle.py)")
    z = np.load(path)
    if f"{name}_epochs" not in z.files:
        pytest.skip(f"no {name} epochs in batched_oracle_thetas.npz yet")
    return {int(e): (th, s) for e, th, s in zip(z[f"{name}_epochs"], z[f"{name}_theta"], z[f"{name}_target_sum"])}


def test_fit_batched_full_uneven_recipe_matches_oracle(dia):
    # the full uneven-batch recipe: 64 epochs of side 512..2048 cut from the shared 2048^2 reference
    # (30,000 stars), 17x17 kernels, one batched fit; every epoch the oracle solved
    # (tests/golden/make_batched_oracle.py: every eighth) against its minimiser at the 1e-4 bar
    gold = _golden("c4")
    b = sf.config4(workers=16)
    m = b.m
    for e, (_, s) in gold.items():
        assert float(np.sum(b.epochs[e].I, dtype=np.float64)) == s, "the seeded inputs differ from the solved ones"
    o, _ = objs(dia, b)
    theta, res, st = dia.fit_batched(gpu(b.R), epochs_gpu(dia, b), m, o)
    th = theta.cpu().double().numpy()
    assert st >= 0 and all(r.status >= 0 for r in res)
    worst = 0.0
    for e, (ref, _) in gold.items():
        K, Kr = th[e, :m * m], ref[:m * m]
        eK = np.linalg.norm(K - Kr) / np.linalg.norm(Kr)
        eP = abs(res[e].P - Kr.sum()) / abs(Kr.sum())
        eB = abs(res[e].B0 - ref[-1]) / max(abs(ref[-1]), 1.0)
        worst = max(worst, eK, eP, eB)
        assert eK <= 1e-4 and eP <= 1e-4 and eB <= 1e-4, (e, b.epochs[e].I.shape, eK, eP, eB)
    print(f"uneven batch: {len(gold)} epochs checked, worst relative error {worst:.2e}")


def test_fit_batched_full_shared_recipe_sample_matches_oracle(dia):
    # eight epochs of the 256 x 2048^2, m = 25 recipe (the first eight the oracle solved), both precisions
    gold = _golden("c5")
    pick = sorted(gold)[:8]
    b = sf.config5(n_epochs=max(pick) + 1, workers=16)
    m = b.m
    eps = [b.epochs[e] for e in pick]
    for e in pick:
        assert float(np.sum(b.epochs[e].I, dtype=np.float64)) == gold[e][1]
    o, _ = objs(dia, b)
    E = [dia.Epoch(I=gpu(ep.I), ref_row0=ep.row0, ref_col0=ep.col0) for ep in eps]
    for prec in ("plain", "bf16x3"):
        theta, res, st = dia.fit_batched(gpu(b.R), E, m, o, precision=prec)
        th = theta.cpu().double().numpy()
        assert st >= 0
        for k, e in enumerate(pick):
            ref = gold[e][0]
            K, Kr = th[k, :m * m], ref[:m * m]
            eK = np.linalg.norm(K - Kr) / np.linalg.norm(Kr)
            eP = abs(res[k].P - Kr.sum()) / abs(Kr.sum())
            eB = abs(res[k].B0 - ref[-1]) / max(abs(ref[-1]), 1.0)
            assert eK <= 1e-4 and eP <= 1e-4 and eB <= 1e-4, (prec, e, eK, eP, eB)
