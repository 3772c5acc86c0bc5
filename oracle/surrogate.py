"""CNN surrogate of the evaluation, plain FP64 reference (test infrastructure).

TEST INFRASTRUCTURE ONLY: used by ``tests/`` and nothing else.

The surrogate maps a pixel map (n_layers x ny x nx, 0/1) and a frequency to
the complex S entries the FoM of Eqs. 8-9 needs most (S11, S21, S31), so that a
search step can rank all candidate flips of Algorithm 1 and solve only the best
few exactly.  It is not in the paper; the architecture is the build's:

    x0  = map as an image, channels = layers              (B, ny, nx, L)
    a1  = relu(conv3x3(x0; W1, b1))                        32 channels
    a2  = pool2(relu(conv3x3(a1; W2, b2)))                 32
    a3  = relu(conv3x3(a2; W3, b3))                        64
    a4  = pool2(relu(conv3x3(a3; W4, b4)))                 64
    feat = a4 flattened in (y, x, channel) order           D = (ny//4)(nx//4) 64
    e(u) = [sin(pi u), cos(pi u), sin(2 pi u), cos(2 pi u), ...]   E values
    h   = relu(feat Wf + e(u) We + bh)                     hidden units
    out = h Wo + bo                                        n_out = 2 x entries (re, im)

conv3x3 has zero padding 1 and weights indexed [tap = 3 dy + dx][c_in][c_out]
acting on x[y + dy - 1, x + dx - 1]; pool2 averages 2 x 2 blocks and drops an
odd last row or column; u = (f - f_lo) / (f_hi - f_lo).  The loss is the mean
squared error over every output of every (map, frequency).  Parameters are one
flat vector in the order of ``layout``.  Training uses AdamW (Loshchilov and
Hutter, "Decoupled weight decay regularization", ICLR 2019) with bias-corrected
moments and the decay applied to every parameter.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class SurrogateConfig:
    n_layers: int
    ny: int
    nx: int
    channels: tuple = (32, 32, 64, 64)
    hidden: int = 256
    emb: int = 16
    n_out: int = 6

    @property
    def feat_dim(self) -> int:
        return (self.ny // 2 // 2) * (self.nx // 2 // 2) * self.channels[3]


def layout(cfg: SurrogateConfig):
    """(name, shape) of every parameter tensor, in flat-vector order."""
    c = (cfg.n_layers,) + tuple(cfg.channels)
    out = []
    for i in range(4):
        out.append((f"W{i + 1}", (9, c[i], c[i + 1])))
        out.append((f"b{i + 1}", (c[i + 1],)))
    out += [("Wf", (cfg.feat_dim, cfg.hidden)), ("We", (cfg.emb, cfg.hidden)), ("bh", (cfg.hidden,)),
            ("Wo", (cfg.hidden, cfg.n_out)), ("bo", (cfg.n_out,))]
    return out


def n_params(cfg: SurrogateConfig) -> int:
    return int(sum(np.prod(s) for _, s in layout(cfg)))


def unpack(params: np.ndarray, cfg: SurrogateConfig) -> dict:
    d, o = {}, 0
    for name, shape in layout(cfg):
        n = int(np.prod(shape))
        d[name] = params[o:o + n].reshape(shape)
        o += n
    return d


def pack(d: dict, cfg: SurrogateConfig) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in layout(cfg)])


def map_image(maps: np.ndarray, cfg: SurrogateConfig) -> np.ndarray:
    """(B, n_cells) 0/1 -> (B, ny, nx, L): cell l*ny*nx + y*nx + x is pixel (y, x) of channel l."""
    B = maps.shape[0]
    return maps.reshape(B, cfg.n_layers, cfg.ny, cfg.nx).transpose(0, 2, 3, 1).astype(np.float64)


def embedding(u: np.ndarray, E: int) -> np.ndarray:
    """(F, E): columns 2j and 2j+1 are sin((j+1) pi u) and cos((j+1) pi u)."""
    u = np.asarray(u, np.float64)
    e = np.empty((len(u), E))
    for j in range(E // 2):
        e[:, 2 * j] = np.sin((j + 1) * np.pi * u)
        e[:, 2 * j + 1] = np.cos((j + 1) * np.pi * u)
    return e


def _shifted(X: np.ndarray, dy: int, dx: int) -> np.ndarray:
    """S[b, y, x, :] = X[b, y + dy - 1, x + dx - 1, :], zero outside the image."""
    B, H, W, C = X.shape
    S = np.zeros_like(X)
    ys, yd = max(0, dy - 1), max(0, 1 - dy)
    xs, xd = max(0, dx - 1), max(0, 1 - dx)
    h, w = H - abs(dy - 1), W - abs(dx - 1)
    S[:, yd:yd + h, xd:xd + w, :] = X[:, ys:ys + h, xs:xs + w, :]
    return S


def conv3x3(X: np.ndarray, Wt: np.ndarray, b: np.ndarray) -> np.ndarray:
    Y = np.broadcast_to(b, X.shape[:3] + (Wt.shape[2],)).copy()
    for dy in range(3):
        for dx in range(3):
            Y += _shifted(X, dy, dx) @ Wt[3 * dy + dx]
    return Y


def conv3x3_backward(X: np.ndarray, Wt: np.ndarray, dY: np.ndarray):
    """Gradients of sum(dY * conv3x3(X)) with respect to X, W and b."""
    dX = np.zeros_like(X)
    dW = np.zeros_like(Wt)
    B, H, W, _ = X.shape
    for dy in range(3):
        for dx in range(3):
            t = 3 * dy + dx
            dW[t] = np.einsum("byxi,byxo->io", _shifted(X, dy, dx), dY)
            # X[y', x'] feeds Y[y' - dy + 1, x' - dx + 1]
            dX += _shifted(dY @ Wt[t].T, 2 - dy, 2 - dx)
    return dX, dW, dY.sum(axis=(0, 1, 2))


def pool2(X: np.ndarray) -> np.ndarray:
    B, H, W, C = X.shape
    h, w = H // 2, W // 2
    Xc = X[:, :2 * h, :2 * w, :]
    return 0.25 * (Xc[:, 0::2, 0::2] + Xc[:, 1::2, 0::2] + Xc[:, 0::2, 1::2] + Xc[:, 1::2, 1::2])


def pool2_backward(shape, dY: np.ndarray) -> np.ndarray:
    dX = np.zeros(shape)
    h, w = dY.shape[1], dY.shape[2]
    for i in range(2):
        for j in range(2):
            dX[:, i:2 * h:2, j:2 * w:2, :] = 0.25 * dY
    return dX


def forward(params: np.ndarray, maps: np.ndarray, u: np.ndarray, cfg: SurrogateConfig):
    """Outputs (B, F, n_out) and the intermediate values the gradient needs."""
    p = unpack(params, cfg)
    x0 = map_image(maps, cfg)
    z1 = conv3x3(x0, p["W1"], p["b1"]); a1 = np.maximum(z1, 0)
    z2 = conv3x3(a1, p["W2"], p["b2"]); a2 = pool2(np.maximum(z2, 0))
    z3 = conv3x3(a2, p["W3"], p["b3"]); a3 = np.maximum(z3, 0)
    z4 = conv3x3(a3, p["W4"], p["b4"]); a4 = pool2(np.maximum(z4, 0))
    feat = a4.reshape(a4.shape[0], -1)
    e = embedding(u, cfg.emb)
    zh = (feat @ p["Wf"])[:, None, :] + (e @ p["We"])[None, :, :] + p["bh"]
    h = np.maximum(zh, 0)
    out = h @ p["Wo"] + p["bo"]
    cache = dict(x0=x0, z1=z1, a1=a1, z2=z2, a2=a2, z3=z3, a3=a3, z4=z4, feat=feat, e=e, zh=zh, h=h)
    return out, cache


def loss(out: np.ndarray, target: np.ndarray) -> float:
    return float(np.mean((out - target) ** 2))


def gradient(params: np.ndarray, maps: np.ndarray, u: np.ndarray, target: np.ndarray, cfg: SurrogateConfig):
    """(loss, d loss / d params) by the chain rule through ``forward``."""
    p = unpack(params, cfg)
    out, k = forward(params, maps, u, cfg)
    g = {}
    dout = 2.0 * (out - target) / out.size
    g["Wo"] = np.einsum("bfh,bfo->ho", k["h"], dout)
    g["bo"] = dout.sum(axis=(0, 1))
    dzh = (dout @ p["Wo"].T) * (k["zh"] > 0)
    g["bh"] = dzh.sum(axis=(0, 1))
    g["Wf"] = k["feat"].T @ dzh.sum(axis=1)
    g["We"] = k["e"].T @ dzh.sum(axis=0)
    dfeat = dzh.sum(axis=1) @ p["Wf"].T
    z4 = k["z4"]
    dz4 = pool2_backward(z4.shape, dfeat.reshape(k["z4"].shape[0], z4.shape[1] // 2, z4.shape[2] // 2, -1)) * (z4 > 0)
    da3, g["W4"], g["b4"] = conv3x3_backward(k["a3"], p["W4"], dz4)
    dz3 = da3 * (k["z3"] > 0)
    da2, g["W3"], g["b3"] = conv3x3_backward(k["a2"], p["W3"], dz3)
    z2 = k["z2"]
    dz2 = pool2_backward(z2.shape, da2) * (z2 > 0)
    da1, g["W2"], g["b2"] = conv3x3_backward(k["a1"], p["W2"], dz2)
    dz1 = da1 * (k["z1"] > 0)
    _, g["W1"], g["b1"] = conv3x3_backward(k["x0"], p["W1"], dz1)
    return loss(out, target), pack(g, cfg)


def adamw_step(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
    """One AdamW update at step t (1-based); returns new (params, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** t)
    vhat = v / (1 - beta2 ** t)
    return params - lr * (mhat / (np.sqrt(vhat) + eps) + weight_decay * params), m, v
