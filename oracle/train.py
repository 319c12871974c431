"""Training oracle: one optimisation step of an LSNIF object, plainly, in float64.

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU baseline
of the benchmark may call this module.  It shares no code with the GPU library.

What one step computes (paper Sec. 5.2 and 5.3):

- the forward pass of each training ray: the voxel walk, the boundary points
  and the encoding come from the query oracle (``oracle.query`` with
  ``debug=True``, float64 features from the float32 tables), then the MLP
  without biases, hidden activations ReLU or leaky ReLU (Sec. 3.3, 5.1);
- the per-signal activations and losses of Sec. 5.3: occlusion by sigmoid and
  binary cross-entropy; local hit distance by sigmoid and mean absolute error
  against the reference distance mapped onto the ray's AABB interval; normal
  by the identity and the cosine-similarity loss; albedo by sigmoid and the
  relative L2 loss of Lehtinen et al. 2018 (squared error over the squared
  output plus 0.01, the output in the denominator held constant); material
  by softmax and categorical cross-entropy.  All non-occlusion terms are zero
  for rays whose reference is a miss (Sec. 5.3);
- the batch loss: the sum of the per-ray losses over the batch size;
- its gradient with respect to every table entry and weight (backward pass,
  written out layer by layer; the encoding is linear in the table entries,
  each point's feature = sum over its cell corners of trilinear weight x
  entry, so an entry's gradient is the sum of weight x d loss / d feature over
  the points that reach it);
- Adam (Kingma and Ba 2015, Algorithm 1), the optimiser Sec. 5.2 names, with
  the paper's learning rate 0.01 and the Adam paper's defaults otherwise.

Readings where the paper is silent, each listed with its reason in the design
notes: the signals' losses are summed with weight 1 and the albedo and normal
terms averaged over their components as stated above; the batch mean is over
all rays of the batch; a ray with no listed voxel adds nothing (its network
input is zero, and a query calls it a miss without running the network); the
cosine similarity divides by max(|z_n|, 1e-8); the activation derivative at 0
and the absolute value's derivative at 0 are taken as the value below 0 and
0; Adam is dense (every parameter every step) with beta1 0.9, beta2 0.999,
eps 1e-8.
"""
import numpy as np

from . import query as _query

ADAM_DEFAULTS = dict(lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8)


def _sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def mlp_forward(obj, enc):
    """Layer inputs (acts[0] = encoding, acts[k] = activated output of hidden layer k)
    and the raw outputs z, float64."""
    slope = float(np.float32(obj.leaky_slope)) if obj.act == 1 else 0.0   # the slope as the object descriptor holds it (float32)
    W = [np.asarray(w, np.float64) for w in obj.weights]
    acts = [np.asarray(enc, np.float64)]
    for k in range(len(W) - 1):
        pre = acts[-1] @ W[k].T
        acts.append(np.where(pre > 0.0, pre, slope * pre))
    return acts, acts[-1] @ W[-1].T


def losses(obj, z, targets, tatb, active, albedo_den=None):
    """Per-ray loss and d (per-ray loss) / d z for raw outputs z (n, out_dim).

    ``targets``: dict with ``hit`` (n,), ``t`` (n,), ``n`` (n, 3), ``albedo`` (n, 3),
    ``material`` (n,).  ``tatb``: the rays' AABB interval.  ``active``: rays with at
    least one listed voxel; the others get loss 0 and gradient 0.  ``albedo_den``: the albedo
    term's denominators (a + 0.01)^2 to hold (default: from z), so that a finite difference
    of the loss sees them as the constants the gradient takes them for.  Also returns the
    denominators used.
    """
    n_rays, od = z.shape
    y = np.asarray(targets["hit"]).astype(bool) & active
    loss = np.zeros(n_rays)
    dz = np.zeros((n_rays, od))
    # occlusion: sigmoid + binary cross-entropy, as softplus(z0) - y z0
    z0 = z[:, 0]
    yh = y.astype(np.float64)
    loss += np.logaddexp(0.0, z0) - yh * z0
    dz[:, 0] = _sigmoid(z0) - yh
    # local hit distance: sigmoid + absolute error against (t - ta) / (tb - ta)
    ta, tb = tatb[:, 0].astype(np.float64), tatb[:, 1].astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        tau = np.clip((np.asarray(targets["t"], np.float64) - ta) / (tb - ta), 0.0, 1.0)
    s1 = _sigmoid(z[:, 1])
    e1 = s1 - tau
    loss += np.where(y, np.abs(e1), 0.0)
    dz[:, 1] = np.where(y, np.sign(e1) * s1 * (1.0 - s1), 0.0)
    # normal: identity + (1 - cosine similarity)
    zn = z[:, 2:5]
    ny = np.asarray(targets["n"], np.float64)
    nn = np.linalg.norm(zn, axis=1)
    den = np.maximum(nn, 1e-8)
    cs = np.sum(zn * ny, axis=1) / den
    loss += np.where(y, 1.0 - cs, 0.0)
    big = nn > 1e-8
    safe = np.where(big, nn, 1.0)
    g_n = np.where(big[:, None], -(ny / safe[:, None] - cs[:, None] * zn / (safe * safe)[:, None]), -ny / 1e-8)
    dz[:, 2:5] = np.where(y[:, None], g_n, 0.0)
    m0 = 5
    if obj.has_albedo:
        a = _sigmoid(z[:, 5:8])
        e = a - np.asarray(targets["albedo"], np.float64)
        q = (a + 0.01) ** 2 if albedo_den is None else albedo_den
        loss += np.where(y, np.mean(e * e / q, axis=1), 0.0)
        dz[:, 5:8] = np.where(y[:, None], (2.0 * e / q) / 3.0 * a * (1.0 - a), 0.0)
        m0 = 8
    # material: softmax + categorical cross-entropy (rays whose index is out of range skip it)
    zm = z[:, m0:m0 + obj.n_mat]
    mat = np.asarray(targets["material"], np.int64)
    ok = y & (mat >= 0) & (mat < obj.n_mat)
    mx = zm.max(axis=1, keepdims=True)
    ex = np.exp(zm - mx)
    lse = mx[:, 0] + np.log(ex.sum(axis=1))
    pick = zm[np.arange(n_rays), np.clip(mat, 0, obj.n_mat - 1)]
    loss += np.where(ok, lse - pick, 0.0)
    onehot = np.zeros_like(zm)
    onehot[np.arange(n_rays), np.clip(mat, 0, obj.n_mat - 1)] = 1.0
    dz[:, m0:m0 + obj.n_mat] = np.where(ok[:, None], ex / ex.sum(axis=1, keepdims=True) - onehot, 0.0)
    loss = np.where(active, loss, 0.0)
    dz[~active] = 0.0
    return loss, dz, (q if obj.has_albedo else None)


def train_grads(obj, rays, targets, bounds=False):
    """Batch loss and its gradients for one batch.

    Returns a dict: ``loss`` (float), ``gtab`` (L, T, F) and ``gW`` (list of [out][in]) in
    float64, ``z`` raw outputs, ``pre_acts`` (the layer inputs), ``active``, ``tatb``,
    ``count``, ``enc``; with ``bounds`` also ``gtab_abs`` and ``gW_abs``, the same sums over absolute
    values of the terms (the scale of each gradient entry's rounding error).
    """
    rays = np.ascontiguousarray(rays, np.float32)
    n = len(rays)
    q = _query(obj, rays, debug=True)
    count = q["count"]
    active = count > 0
    acts, z = mlp_forward(obj, q["enc"])
    z[~active] = 0.0
    loss_r, dz, den = losses(obj, z, targets, q["tatb"], active)
    G = dz / n
    W = [np.asarray(w, np.float64) for w in obj.weights]
    slope = float(np.float32(obj.leaky_slope)) if obj.act == 1 else 0.0   # the slope as the object descriptor holds it (float32)
    gW = [None] * len(W)
    gW_abs = [None] * len(W)
    Gabs = np.abs(G)
    for k in range(len(W) - 1, -1, -1):
        gW[k] = G.T @ acts[k]
        if bounds:
            gW_abs[k] = Gabs.T @ np.abs(acts[k])
        gin = G @ W[k]
        if bounds:
            gin_abs = Gabs @ np.abs(W[k])
        if k > 0:
            d = np.where(acts[k] > 0.0, 1.0, slope)
            G = gin * d
            if bounds:
                Gabs = gin_abs * d
        else:
            G = gin
            if bounds:
                Gabs = gin_abs
    # the encoding's transpose: scatter d loss / d feature onto the table entries
    H, L, F = obj.H, obj.L, obj.F
    dx = G.reshape(n, H, L, F)
    h_idx = np.arange(H)[None, :]
    live = (h_idx < count[:, None])                               # (n, H) points that exist
    wt = q["weights"].astype(np.float64)                          # (n, H, L, 3)
    slots = q["slots"].astype(np.int64)                           # (n, H, L, 8)
    T = 1 << obj.log2_T
    gtab = np.zeros((L, T, F))
    gtab_abs = np.zeros((L, T, F)) if bounds else None
    absdx = Gabs.reshape(n, H, L, F) if bounds else None
    for c in range(8):
        wc = np.ones(wt.shape[:3])
        for b in range(3):
            wc = wc * (wt[..., b] if (c >> b) & 1 else 1.0 - wt[..., b])
        contrib = wc[..., None] * dx                              # (n, H, L, F)
        for l in range(L):
            idx = slots[:, :, l, c][live]
            for f in range(F):
                np.add.at(gtab[l, :, f], idx, contrib[:, :, l, f][live])
                if bounds:
                    np.add.at(gtab_abs[l, :, f], idx, (np.abs(wc[:, :, l]) * absdx[:, :, l, f])[live])
    out = {"loss": float(loss_r.sum() / n), "loss_r": loss_r, "gtab": gtab, "gW": gW, "z": z,
           "pre_acts": acts, "active": active, "tatb": q["tatb"], "count": count, "enc": q["enc"],
           "albedo_den": den}
    if bounds:
        out["gtab_abs"] = gtab_abs
        out["gW_abs"] = gW_abs
    return out


def batch_loss(obj, rays, targets, albedo_den=None):
    """The batch loss alone (the forward pass of ``train_grads``), optionally with the
    albedo denominators held at given values."""
    rays = np.ascontiguousarray(rays, np.float32)
    q = _query(obj, rays, debug=True)
    active = q["count"] > 0
    _, z = mlp_forward(obj, q["enc"])
    z[~active] = 0.0
    loss_r, _, _ = losses(obj, z, targets, q["tatb"], active, albedo_den)
    return float(loss_r.sum() / len(rays))


def adam(p, g, m, v, t, lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step at step number t (1-based): returns (p, m, v), float64."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
