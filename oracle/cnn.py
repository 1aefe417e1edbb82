"""FP64 reference of the warm-start network (test infrastructure).

Four 3x3 convolutions with "same" zero padding: C_in -> 32 -> 32 -> 32 -> 1,
dilations DIL = (1, 2, 4, 8) (tap (dy, dx) reads the pixel d*(dy, dx) away;
receptive field 31 pixels), ReLU after the first three, biases in FP32/FP64.
Activations are NHWC.  The
arithmetic is FP64; the values that the device keeps in BF16 are rounded to
BF16 (round to nearest even) at the same points:
  * the input tensor x0 and every weight tensor used by a convolution,
  * the stored activations y1, y2, y3 (after bias and ReLU),
  * the back-propagated pre-activation gradients g1, g2, g3 (inputs of the
    matrix-core products).
The loss gradient g4 and the last layer's products stay in full precision.
Weight layout: W[l] has shape (C_out, 3, 3, C_in) (tap (dy, dx) in row-major
order, dy, dx in {-1, 0, 1}); b[l] has shape (C_out,).

Loss: mean squared error over the masked pixels of every sample,
L = sum_{b, p in mask} (out - target)^2 / (B * |mask|).
"""
from __future__ import annotations

import numpy as np

CH = 32
DIL = (1, 2, 4, 8)


def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    a = np.asarray(x, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(a)
    if nan.any():
        out[nan] = np.nan
    return out


def init_params(c_in=4, seed=0):
    """He-normal weights, zero biases (FP32 master values, as float64 arrays)."""
    rng = np.random.default_rng(seed)
    shapes = [(CH, 3, 3, c_in), (CH, 3, 3, CH), (CH, 3, 3, CH), (1, 3, 3, CH)]
    W, b = [], []
    for s in shapes:
        fan_in = 9 * s[3]
        W.append((rng.standard_normal(s) * np.sqrt(2.0 / fan_in)).astype(np.float32).astype(np.float64))
        b.append(np.zeros(s[0]))
    return W, b


def _shift(x, oy, ox):
    """x shifted so that out[y, x] = x[y + oy, x + ox] (zero outside)."""
    B, H, Wd, C = x.shape
    out = np.zeros_like(x)
    ys, ye = max(0, -oy), min(H, H - oy)
    xs, xe = max(0, -ox), min(Wd, Wd - ox)
    if ys < ye and xs < xe:
        out[:, ys:ye, xs:xe] = x[:, ys + oy:ye + oy, xs + ox:xe + ox]
    return out


def conv(x, Wt, bias, d=1):
    """z[b,y,x,n] = sum_{dy,dx,c} W[n,dy+1,dx+1,c] x[b,y+d*dy,x+d*dx,c] + bias[n] (zero padding)."""
    z = np.zeros(x.shape[:3] + (Wt.shape[0],))
    for dy in range(3):
        for dx in range(3):
            z += _shift(x, d * (dy - 1), d * (dx - 1)) @ Wt[:, dy, dx, :].T
    return z + bias


def conv_transpose(g, Wt, d=1):
    """dL/dx for z = conv(x, W, d): dx[p] = sum_{tap,n} W[n,tap,c] g[p - d*off(tap), n]."""
    dx_ = np.zeros(g.shape[:3] + (Wt.shape[3],))
    for dy in range(3):
        for dx in range(3):
            dx_ += _shift(g, -d * (dy - 1), -d * (dx - 1)) @ Wt[:, dy, dx, :]
    return dx_


def conv_wgrad(g, x, d=1):
    """dL/dW[n,dy,dx,c] = sum_{b,p} g[b,p,n] x[b,p+d*(dy-1,dx-1),c]; dL/db[n] = sum g."""
    N = g.shape[3]
    C = x.shape[3]
    dW = np.zeros((N, 3, 3, C))
    gf = g.reshape(-1, N)
    for dy in range(3):
        for dx in range(3):
            dW[:, dy, dx, :] = gf.T @ _shift(x, d * (dy - 1), d * (dx - 1)).reshape(-1, C)
    return dW, gf.sum(axis=0)


def forward(x0, W, b, rounding=True):
    """Returns the FP64 output (B,H,W) and the stored activations."""
    r = bf16 if rounding else (lambda v: np.asarray(v, np.float64))
    x = r(x0)
    acts = [x]
    for l in range(3):
        z = conv(x, r(W[l]), b[l], DIL[l])
        x = r(np.maximum(z, 0.0))
        acts.append(x)
    out = conv(x, r(W[3]), b[3], DIL[3])[..., 0]
    return out, acts


def loss_and_grads(x0, target, mask, W, b, rounding=True):
    """MSE loss over masked pixels and its gradients (list dW, list db)."""
    r = bf16 if rounding else (lambda v: np.asarray(v, np.float64))
    out, acts = forward(x0, W, b, rounding)
    B = out.shape[0]
    m = np.broadcast_to(mask, out.shape).astype(np.float64)
    cnt = B * mask.sum()
    diff = (out - target) * m
    loss = float((diff ** 2).sum() / cnt)
    g = (2.0 * diff / cnt)[..., None]  # dL/dz4, (B,H,W,1)
    dW = [None] * 4
    db = [None] * 4
    for l in (3, 2, 1, 0):
        dW[l], db[l] = conv_wgrad(g, acts[l], DIL[l])
        if l == 0:
            break
        dy = conv_transpose(g, r(W[l]), DIL[l])
        g = r(dy * (acts[l] > 0))
    return loss, dW, db, out


def adam(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on a list of arrays; state = (m, v, t)."""
    m, v, t = state
    t += 1
    out = []
    for k, (p, g) in enumerate(zip(params, grads)):
        m[k] = b1 * m[k] + (1 - b1) * g
        v[k] = b2 * v[k] + (1 - b2) * g * g
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        out.append(p - lr * mh / (np.sqrt(vh) + eps))
    return out, (m, v, t)


def pack_inputs(f, s, mask, mu):
    """Network input for B images (f, s: (B,H,W) FP64; mask (H,W); mu (B,)).

    Channels: f/|f|_inf, log10(mu) + 2, s/|s|_inf, mask (norms over masked
    pixels; 1 if zero).  Returned BF16-rounded, with the per-image |s|_inf.
    """
    B, H, W = f.shape
    m = mask.astype(bool)
    x = np.zeros((B, H, W, 4))
    sn = np.zeros(B)
    for b in range(B):
        fn = np.abs(f[b][m]).max() if m.any() else 0.0
        snb = np.abs(s[b][m]).max() if m.any() else 0.0
        fn = fn if fn > 0 else 1.0
        snb = snb if snb > 0 else 1.0
        sn[b] = snb
        x[b, ..., 0] = np.where(m, f[b] / fn, 0.0)
        x[b, ..., 1] = np.log10(mu[b]) + 2.0
        x[b, ..., 2] = np.where(m, s[b] / snb, 0.0)
        x[b, ..., 3] = m
    return bf16(x), sn


def target(u_star, s, sn, mask):
    """(u* - s)/|s|_inf on masked pixels (FP32 values)."""
    t = np.where(mask[None].astype(bool), (u_star - s) / sn[:, None, None], 0.0)
    return np.asarray(t, np.float32).astype(np.float64)


def warm_start(s, sn, out, mask):
    """u = s + |s|_inf * out on masked pixels, 0 elsewhere."""
    return np.where(mask[None].astype(bool), s + sn[:, None, None] * out, 0.0)


def flatten(W, b):
    """Parameters in the device's flat FP32 layout (W1,b1,W2,b2,W3,b3,W4,b4)."""
    return np.concatenate([np.concatenate([w.ravel(), bb.ravel()]) for w, bb in zip(W, b)]).astype(np.float32)


def unflatten(p, c_in=4):
    shapes = [(CH, 3, 3, c_in), (CH, 3, 3, CH), (CH, 3, 3, CH), (1, 3, 3, CH)]
    W, b, o = [], [], 0
    for s in shapes:
        n = int(np.prod(s))
        W.append(np.asarray(p[o:o + n], np.float64).reshape(s))
        o += n
        b.append(np.asarray(p[o:o + s[0]], np.float64))
        o += s[0]
    return W, b
