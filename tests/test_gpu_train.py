"""The GPU training step against the training oracle (paper Sec. 5.2, 5.3).

Tolerances, from the float32 arithmetic of the GPU side:
- batch loss: relative 1e-5 (per-ray float32 losses, summed in float64);
- gradients, per entry: |g_gpu - g_oracle| <= 1e-4 x the oracle's sum of the absolute
  values of the entry's terms (float32 sums of at most a few thousand terms, each from
  float32 forward and backward values that are within ~1e-5 of the float64 ones);
- the ReLU / leaky-ReLU derivative and the sign of the distance error are decisions:
  rays where any hidden pre-activation lies within 2e-5 x sum |w| |x| of 0 (a bound on
  the float32 forward error), or |sigmoid(z1) - tau| < 1e-5, are left out of the batch
  on both sides, so both take the same decisions;
- Adam, given the GPU's own gradients: |p_gpu - p_oracle| <= lr c1 8 u (b1 |m_prev| + (1 - b1)
  |g|) / (sqrt(v_hat) + eps) + 1e-6 |update| + 2 ulp(p), u = 2^-24 (the first moment can cancel,
  so its rounding is bounded by its terms' magnitude, not by its value).
"""
import dataclasses

import numpy as np
import pytest

import oracle
import oracle.train as OT
import workloads as W
from workloads import train as WT

pytestmark = pytest.mark.gpu

F32 = lambda x: float(np.float32(x))
ADAM = dict(lr=F32(0.01), beta1=F32(0.9), beta2=F32(0.999), eps=F32(1e-8))


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2504_21627_amd import lsnif
    return lsnif


@pytest.fixture(scope="module")
def mesh():
    return W.icosphere(3)


def objects():
    return {"paper": W.configs.paper_object(seed=11), "c1": W.configs.c1_object(seed=2)}


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def margin_keep(obj, rays, tg):
    """Rays whose float32 decisions (activation derivative, distance-error sign) are certain."""
    g = OT.train_grads(obj, rays, tg)
    W64 = [np.asarray(w, np.float64) for w in obj.weights]
    keep = np.ones(len(rays), bool)
    acts = g["pre_acts"]
    for k in range(len(W64) - 1):
        pre = acts[k] @ W64[k].T
        bound = np.abs(acts[k]) @ np.abs(W64[k]).T
        keep &= np.all(np.abs(pre) > 2e-5 * bound, axis=1) | ~g["active"]
    ta, tb = g["tatb"][:, 0].astype(np.float64), g["tatb"][:, 1].astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        tau = np.clip((tg["t"].astype(np.float64) - ta) / (tb - ta), 0, 1)
    s1 = 1.0 / (1.0 + np.exp(-g["z"][:, 1]))
    y = (tg["hit"] == 1) & g["active"]
    keep &= ~(y & (np.abs(s1 - tau) < 1e-5))
    return keep


def subset(rays, tg, keep):
    return rays[keep], {k: v[keep] for k, v in tg.items()}


def gpu_grads(L, obj, rays, tg):
    import torch
    ctx = L.lsnif_create(0)
    try:
        oid = L.lsnif_build(ctx, L.ObjectDesc(obj, "fp32", "fp32"))
        tr = L.lsnif_trainer_create(ctx, oid, **ADAM)
        try:
            loss = torch.zeros(1, dtype=torch.float32, device="cuda")
            t = L.targets_array(tg["hit"], tg["t"], tg["n"], tg["material"], tg["albedo"])
            L.lsnif_train_grads(tr, dev(rays), dev(t), loss)
            torch.cuda.synchronize()
            tab, Ws, gtab, gW, steps = L.lsnif_trainer_read(tr, obj)
            return float(loss.item()), gtab, gW, tab, Ws, steps
        finally:
            L.lsnif_trainer_destroy(tr)
    finally:
        L.lsnif_destroy(ctx)


def check_grad(gpu, ref, ref_abs, what):
    err = np.abs(gpu.astype(np.float64) - ref)
    tol = 1e-4 * ref_abs + 1e-30
    bad = err > tol
    assert not bad.any(), (what, int(bad.sum()), float(err[bad].max()), float(tol[bad][np.argmax(err[bad])]))


@pytest.mark.parametrize("which", ["paper", "c1"])
def test_train_grads_match_oracle(L, mesh, which):
    obj = objects()[which]
    rays, tg = WT.batch(mesh, obj, 3000, seed=21)
    keep = margin_keep(obj, rays, tg)
    print(which, "rays kept", int(keep.sum()), "of", len(keep), flush=True)
    assert keep.mean() > 0.7
    rays, tg = subset(rays, tg, keep)
    ref = OT.train_grads(obj, rays, tg, bounds=True)
    loss, gtab, gW, tab, Ws, steps = gpu_grads(L, obj, rays, tg)
    assert abs(loss - ref["loss"]) <= 1e-5 * ref["loss"], (loss, ref["loss"])
    check_grad(gtab, ref["gtab"], ref["gtab_abs"], "tables")
    assert np.count_nonzero(ref["gtab"]) > 1000
    for k in range(len(gW)):
        check_grad(gW[k], ref["gW"][k], ref["gW_abs"][k], f"layer {k}")
    # the gradient pass leaves the parameters alone
    assert np.array_equal(tab, obj.tables) and steps == 0
    for a, b in zip(Ws, obj.weights):
        assert np.array_equal(a, b)


def test_adam_matches_oracle(L, mesh):
    import torch
    obj = objects()["paper"]
    rays, tg = WT.batch(mesh, obj, 2000, seed=22)
    ctx = L.lsnif_create(0)
    try:
        oid = L.lsnif_build(ctx, L.ObjectDesc(obj, "fp32", "fp32"))
        tr = L.lsnif_trainer_create(ctx, oid, **ADAM)
        try:
            loss = torch.zeros(1, dtype=torch.float32, device="cuda")
            drays = dev(rays)
            dt = dev(L.targets_array(tg["hit"], tg["t"], tg["n"], tg["material"], tg["albedo"]))
            m = v = None
            for step in (1, 2):
                L.lsnif_train_grads(tr, drays, dt, loss)
                p0, W0, g_t, g_W, _ = L.lsnif_trainer_read(tr, obj)
                L.lsnif_train_apply(tr)
                p1, W1, _, _, steps = L.lsnif_trainer_read(tr, obj)
                assert steps == step
                params0 = np.concatenate([p0.ravel()] + [w.ravel() for w in W0]).astype(np.float64)
                grads = np.concatenate([g_t.ravel()] + [w.ravel() for w in g_W]).astype(np.float64)
                params1 = np.concatenate([p1.ravel()] + [w.ravel() for w in W1]).astype(np.float64)
                if m is None:
                    m = np.zeros_like(params0)
                    v = np.zeros_like(params0)
                m_prev = m
                want, m, v = OT.adam(params0, grads, m, v, step, **ADAM)
                # float32 rounding: the first moment to within 8 ulp of its terms' magnitude (it
                # may cancel), the rest of the update to 1e-6 relative, the new value to 2 ulp
                b1, lr, eps = ADAM["beta1"], ADAM["lr"], ADAM["eps"]
                c1 = 1.0 / (1.0 - b1 ** step)
                vh = v / (1.0 - ADAM["beta2"] ** step)
                mag_m = b1 * np.abs(m_prev) + (1.0 - b1) * np.abs(grads)
                upd = np.abs(want - params0)
                ulp = np.spacing(np.abs(want).astype(np.float32)).astype(np.float64)
                tol = lr * c1 * 8 * 2.0 ** -24 * mag_m / (np.sqrt(vh) + eps) + 1e-6 * upd + 2 * ulp
                err = np.abs(params1 - want)
                assert np.all(err <= tol), (step, float(err.max()), float((err / tol).max()))
                assert np.count_nonzero(grads) > 1000 and np.all(params1[grads == 0] == params0[grads == 0])
        finally:
            L.lsnif_trainer_destroy(tr)
    finally:
        L.lsnif_destroy(ctx)


def test_training_lowers_loss_and_queries_see_it(L, mesh):
    """Steps on one batch lower its loss; the object answers queries with the trained
    parameters (the FP32 query path against the query oracle on the parameters read back)."""
    import torch
    obj = objects()["paper"]
    rays, tg = WT.batch(mesh, obj, 1 << 14, seed=23)
    ctx = L.lsnif_create(0)
    try:
        oid = L.lsnif_build(ctx, L.ObjectDesc(obj, "fp32", "fp32"))
        tr = L.lsnif_trainer_create(ctx, oid)
        try:
            drays = dev(rays)
            dt = dev(L.targets_array(tg["hit"], tg["t"], tg["n"], tg["material"], tg["albedo"]))
            losses = []
            loss = torch.zeros(1, dtype=torch.float32, device="cuda")
            for _ in range(8):
                L.lsnif_train_step(tr, drays, dt, loss)
                losses.append(float(loss.item()))
            print("losses", losses, flush=True)
            assert all(b < a for a, b in zip(losses, losses[1:])) and losses[-1] < 0.8 * losses[0]
            tab, Ws, _, _, steps = L.lsnif_trainer_read(tr, obj)
            assert steps == 8
            out = torch.empty((len(rays), 6), dtype=torch.float32, device="cuda")
            L.lsnif_query(ctx, oid, drays, out)
            torch.cuda.synchronize()
            g = out.cpu().numpy()
            trained = dataclasses.replace(obj, tables=tab, weights=Ws)
            o = oracle.query(trained, rays)
            cand = o["count"] > 0
            agree = (g[:, 0].view(np.uint32) == o["hit"])[cand].mean()
            assert agree >= 0.999, agree
            # training on: the loss keeps falling, and the object learns to call reference
            # hits hits (printed for the record)
            for _ in range(192):
                L.lsnif_train_step(tr, drays, dt, loss)
            torch.cuda.synchronize()
            print("loss after 200 steps", float(loss.item()), flush=True)
            assert float(loss.item()) < 0.8 * losses[-1]
            out200 = torch.empty((len(rays), 6), dtype=torch.float32, device="cuda")
            L.lsnif_query(ctx, oid, drays, out200)
            torch.cuda.synchronize()
            h200 = out200.cpu().numpy()[:, 0].view(np.uint32)
            y = tg["hit"] == 1
            print("hit recall", float((h200[y] == 1).mean()), "precision",
                  float(y[h200 == 1].mean()) if (h200 == 1).any() else None, flush=True)
        finally:
            L.lsnif_trainer_destroy(tr)
    finally:
        L.lsnif_destroy(ctx)


def test_train_edge_cases(L, mesh):
    import torch
    obj = objects()["c1"]
    ctx = L.lsnif_create(0)
    try:
        oid = L.lsnif_build(ctx, L.ObjectDesc(obj, "fp32", "fp32"))
        half = L.lsnif_build(ctx, L.ObjectDesc(obj, "fp16", "fp16"))
        with pytest.raises(L.LsnifError):
            L.lsnif_trainer_create(ctx, half)
        with pytest.raises(L.LsnifError):
            L.lsnif_trainer_create(ctx, oid, lr=0.0)
        tr = L.lsnif_trainer_create(ctx, oid)
        try:
            loss = torch.zeros(1, dtype=torch.float32, device="cuda")
            # rays that list no voxel: loss 0 and every gradient 0
            far = W.ray_array(np.tile([[5.0, 0.0, 0.0]], (300, 1)), np.tile([[1.0, 0.0, 0.0]], (300, 1)))
            t = L.targets_array(np.ones(300), np.ones(300), np.tile([[1.0, 0, 0]], (300, 1)), np.zeros(300))
            L.lsnif_train_grads(tr, dev(far), dev(t), loss)
            _, _, gtab, gW, _ = L.lsnif_trainer_read(tr, obj)
            assert loss.item() == 0.0 and not gtab.any() and not any(w.any() for w in gW)
            # one ray
            rays, tg = WT.batch(mesh, obj, 64, seed=24)
            i = int(np.argmax(tg["hit"]))
            r1, t1 = rays[i:i + 1], {k: v[i:i + 1] for k, v in tg.items()}
            ref = OT.train_grads(obj, r1, t1, bounds=True)
            L.lsnif_train_grads(tr, dev(r1), dev(L.targets_array(t1["hit"], t1["t"], t1["n"], t1["material"])), loss)
            _, _, gtab, gW, _ = L.lsnif_trainer_read(tr, obj)
            assert abs(loss.item() - ref["loss"]) <= 1e-5 * ref["loss"]
            check_grad(gtab, ref["gtab"], ref["gtab_abs"], "tables, one ray")
            # an empty batch is an error
            with pytest.raises(L.LsnifError):
                L.lsnif_train_grads(tr, dev(far[:0]), dev(t[:0]), loss)
        finally:
            L.lsnif_trainer_destroy(tr)
        # a released object: the trainer refuses
        tr = L.lsnif_trainer_create(ctx, oid)
        L.lsnif_release(ctx, oid)
        with pytest.raises(L.LsnifError):
            L.lsnif_train_apply(tr)
        L.lsnif_trainer_destroy(tr)
    finally:
        L.lsnif_destroy(ctx)


def random_targets(rays, seed, n_mat):
    """Seeded targets of any value (gradient parity does not need them to be geometric):
    a quarter of the rays hit at t in [0, 4], unit normals, materials and albedos."""
    rng = np.random.default_rng(seed)
    n = len(rays)
    nrm = rng.standard_normal((n, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return {"hit": (rng.random(n) < 0.25).astype(np.uint32), "t": rng.uniform(0, 4, n).astype(np.float32),
            "n": nrm.astype(np.float32), "albedo": rng.random((n, 3)).astype(np.float32),
            "material": rng.integers(0, n_mat, n).astype(np.int32)}


def test_train_grads_match_oracle_c2_object(L):
    """c2's object: 16 levels (10 hashed, one face-aligned), 2^19 entries x 2 features, 576
    inputs (18 K slices of the first product), 64 MiB of table gradient per copy."""
    obj = W.configs.c2_object()
    rays = W.configs.subsample(W.configs.c2_rays(), 1500, seed=41)
    tg = random_targets(rays, 42, obj.n_mat)
    keep = margin_keep(obj, rays, tg)
    print("c2 rays kept", int(keep.sum()), "of", len(keep), flush=True)
    assert keep.mean() > 0.7
    rays, tg = subset(rays, tg, keep)
    ref = OT.train_grads(obj, rays, tg, bounds=True)
    loss, gtab, gW, _, _, _ = gpu_grads(L, obj, rays, tg)
    assert abs(loss - ref["loss"]) <= 1e-5 * ref["loss"], (loss, ref["loss"])
    check_grad(gtab, ref["gtab"], ref["gtab_abs"], "tables")
    assert np.count_nonzero(ref["gtab"]) > 10000
    for k in range(len(gW)):
        check_grad(gW[k], ref["gW"][k], ref["gW_abs"][k], f"layer {k}")
