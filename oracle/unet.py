"""2D U-Net initializer: forward, backward, loss and Adam step (oracle, FP64; test
infrastructure only).

The paper starts the iteration from a ramp-filtered back-projection (Sec. 2.2) and
calls initialisation a lever on iteration count (Sec. 3.2); the learned start here maps
that FBP image to an image close to the converged reconstruction.  The network is a
plain U-Net (Ronneberger et al. 2015), fixed as follows:

* input u = fbp / s (s: a scale given by the caller), one channel;
* levels l = 0..L-1 with C_l = C 2^l channels at resolution H/2^l x W/2^l;
* encoder: level 0: E0a = relu(conv(u)), E0 = relu(conv(E0a)); level l >= 1:
  P_l = avgpool2(E_{l-1}), E_la = relu(conv(P_l)), E_l = relu(conv(E_la));
* decoder, l = L-2..0: D_{L-1} = E_{L-1}; cat_l = [up2(D_{l+1}), E_l] (channels of the
  upsampled map first), D_la = relu(conv(cat_l)), D_l = relu(conv(D_la));
* head: r = sum_c w_c D_0[c] + b (1x1 convolution), output x0 = fbp + s r;
* every conv is 3x3, zero padding, stride 1, with bias; avgpool2 averages 2x2 blocks;
  up2 repeats each pixel 2x2 (nearest).
* loss = mean over pixels of (r - (target - fbp)/s)^2, i.e. mean((x0 - target)^2)/s^2.

Parameter vector (float32, the interface shared with the library): for each 3x3 conv in
the order E0a, E0b, E1a, E1b, ..., E(L-1)b, D(L-2)a, D(L-2)b, ..., D0a, D0b: weights
[Cout][3][3][Cin] then bias [Cout]; then the head weights [C] and bias [1].

Arrays are NHWC: [B][H][W][C].  With `bf16=True` the oracle rounds to bfloat16 at the
points where the GPU stores or multiplies in bfloat16 (conv weights of every layer but
the first, every stored activation and activation gradient), so that a comparison
isolates accumulation order; `bf16=False` is the exact FP64 network.
"""
from __future__ import annotations

import dataclasses

import numpy as np


# ---------------------------------------------------------------- rounding to bfloat16
def to_bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even) via float32; returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u.astype(np.uint32)).view(np.float32).astype(np.float64)


# ------------------------------------------------------------------------ architecture
@dataclasses.dataclass(frozen=True)
class Arch:
    levels: int = 4
    base: int = 32

    def ch(self, l: int) -> int:
        return self.base * (1 << l)

    def convs(self) -> list:
        """(name, cin, cout) of every 3x3 conv in parameter order."""
        out = []
        for l in range(self.levels):
            cin = 1 if l == 0 else self.ch(l - 1)
            out.append((f"E{l}a", cin, self.ch(l)))
            out.append((f"E{l}b", self.ch(l), self.ch(l)))
        for l in range(self.levels - 2, -1, -1):
            out.append((f"D{l}a", self.ch(l + 1) + self.ch(l), self.ch(l)))
            out.append((f"D{l}b", self.ch(l), self.ch(l)))
        return out

    def n_params(self) -> int:
        n = sum(co * 9 * ci + co for _, ci, co in self.convs())
        return n + self.base + 1


def unpack(arch: Arch, theta: np.ndarray) -> dict:
    """Split the flat parameter vector into {name: (W [Cout,3,3,Cin], b [Cout])}."""
    theta = np.asarray(theta, dtype=np.float64)
    p, o = {}, 0
    for name, ci, co in arch.convs():
        w = theta[o:o + co * 9 * ci].reshape(co, 3, 3, ci)
        o += co * 9 * ci
        b = theta[o:o + co]
        o += co
        p[name] = (w, b)
    p["head"] = (theta[o:o + arch.base], theta[o + arch.base])
    assert o + arch.base + 1 == theta.size
    return p


def pack(arch: Arch, p: dict) -> np.ndarray:
    parts = []
    for name, _, _ in arch.convs():
        parts += [p[name][0].ravel(), np.ravel(p[name][1])]
    parts += [np.ravel(p["head"][0]), np.ravel(p["head"][1])]
    return np.concatenate(parts)


def init_params(arch: Arch, seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases; head scaled by 0.1."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, ci, co in arch.convs():
        p[name] = (rng.standard_normal((co, 3, 3, ci)) * np.sqrt(2.0 / (9 * ci)), np.zeros(co))
    p["head"] = (0.1 * rng.standard_normal(arch.base) * np.sqrt(1.0 / arch.base), np.zeros(1))
    return pack(arch, p).astype(np.float32).astype(np.float64)


# -------------------------------------------------------------------------- operations
def conv3x3(x: np.ndarray, w: np.ndarray, b) -> np.ndarray:
    """y[n,i,j,o] = b[o] + sum_{ky,kx,c} w[o,ky,kx,c] x[n,i+ky-1,j+kx-1,c], zero padding."""
    n, h, wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    y = np.zeros((n, h, wd, w.shape[0]))
    for ky in range(3):
        for kx in range(3):
            y += xp[:, ky:ky + h, kx:kx + wd, :] @ w[:, ky, kx, :].T
    return y + (0.0 if b is None else np.asarray(b))


def conv3x3_dgrad(dy: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Gradient of sum(dy * conv3x3(x, w, .)) with respect to x."""
    n, h, wd, _ = dy.shape
    dx = np.zeros((n, h + 2, wd + 2, w.shape[3]))
    for ky in range(3):
        for kx in range(3):
            dx[:, ky:ky + h, kx:kx + wd, :] += dy @ w[:, ky, kx, :]
    return dx[:, 1:-1, 1:-1, :]


def conv3x3_wgrad(dy: np.ndarray, x: np.ndarray):
    """Gradients of sum(dy * conv3x3(x, w, b)) with respect to w [Cout,3,3,Cin] and b."""
    n, h, wd, ci = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dw = np.zeros((dy.shape[3], 3, 3, ci))
    d2 = dy.reshape(-1, dy.shape[3])
    for ky in range(3):
        for kx in range(3):
            dw[:, ky, kx, :] = d2.T @ xp[:, ky:ky + h, kx:kx + wd, :].reshape(-1, ci)
    return dw, d2.sum(axis=0)


def avgpool2(x: np.ndarray) -> np.ndarray:
    n, h, w, c = x.shape
    return x.reshape(n, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4))


def avgpool2_back(dy: np.ndarray) -> np.ndarray:
    return 0.25 * up2(dy)


def up2(x: np.ndarray) -> np.ndarray:
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_back(dy: np.ndarray) -> np.ndarray:
    n, h, w, c = dy.shape
    return dy.reshape(n, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4))


def relu(x):
    return np.maximum(x, 0.0)


# ------------------------------------------------------------------- forward, backward
def forward(arch: Arch, theta: np.ndarray, fbp: np.ndarray, s: float, bf16: bool = False):
    """Returns (x0 [B,H,W], r [B,H,W], cache) for fbp [B,H,W]."""
    q = to_bf16 if bf16 else (lambda a: a)
    p = unpack(arch, theta)
    L = arch.levels
    u = (np.asarray(fbp, dtype=np.float64) / s)[..., None]
    c = {"u": u}

    def layer(name, x, first=False):
        w, b = p[name]
        return q(relu(conv3x3(x, w if first else q(w), b)))

    E = []
    x = u
    for l in range(L):
        if l > 0:
            x = q(avgpool2(E[l - 1]))
            c[f"P{l}"] = x
        a = layer(f"E{l}a", x, first=(l == 0))
        c[f"E{l}a"] = a
        e = layer(f"E{l}b", a)
        c[f"E{l}"] = e
        E.append(e)
    d = E[L - 1]
    for l in range(L - 2, -1, -1):
        cat = np.concatenate([up2(d), E[l]], axis=3)
        c[f"cat{l}"] = cat
        a = layer(f"D{l}a", cat)
        c[f"D{l}a"] = a
        d = layer(f"D{l}b", a)
        c[f"D{l}"] = d
    hw, hb = p["head"]
    r = d @ hw + hb
    c["r"] = r
    return np.asarray(fbp) + s * r, r, c


def loss_and_grad(arch: Arch, theta: np.ndarray, fbp: np.ndarray, target: np.ndarray, s: float,
                  bf16: bool = False):
    """(loss, dtheta) with loss = mean((r - (target - fbp)/s)^2)."""
    q = to_bf16 if bf16 else (lambda a: a)
    p = unpack(arch, theta)
    L = arch.levels
    _, r, c = forward(arch, theta, fbp, s, bf16)
    t = (np.asarray(target, dtype=np.float64) - np.asarray(fbp, dtype=np.float64)) / s
    npx = r.size
    diff = r - t
    loss = float(np.mean(diff ** 2))
    dr = 2.0 * diff / npx
    g = {}
    hw, _ = p["head"]
    d_last = c["D0"] if L > 1 else c["E0"]
    g["head"] = ((d_last * dr[..., None]).reshape(-1, arch.base).sum(axis=0), np.array([dr.sum()]))
    # gradient with respect to the pre-activation of the layer producing `out`
    dz = q(dr[..., None] * hw[None, None, None, :] * (d_last > 0))

    def back(name, dz, x, mask_input, first=False):
        w, _ = p[name]
        dw, db = conv3x3_wgrad(dz, x)
        g[name] = (dw, db)
        if first:
            return None
        dx = conv3x3_dgrad(dz, q(w))
        if mask_input:
            dx = dx * (x > 0)
        return dx

    dE = [None] * L  # gradient w.r.t. E_l (masked), filled by the skip and the pooling paths
    for l in range(0, L - 1):
        # decoder level l, traversed from the head upwards: D_l <- D_la <- cat_l
        da = q(back(f"D{l}b", dz, c[f"D{l}a"], True))
        dcat = q(back(f"D{l}a", da, c[f"cat{l}"], True))
        cu = arch.ch(l + 1)
        dE[l] = dcat[..., cu:]
        dz = q(up2_back(dcat[..., :cu]))  # gradient at the pre-activation of D_{l+1} (masked)
    # dz now belongs to E_{L-1} (= D_{L-1})
    for l in range(L - 1, -1, -1):
        dzl = dz if l == L - 1 else dE[l]
        da = q(back(f"E{l}b", dzl, c[f"E{l}a"], True))
        x_in = c["u"] if l == 0 else c[f"P{l}"]
        dp = back(f"E{l}a", da, x_in, False, first=(l == 0))
        if l > 0:
            dp = q(dp)
            dE[l - 1] = q(dE[l - 1] + avgpool2_back(dp) * (c[f"E{l - 1}"] > 0))
    grads = {k: v for k, v in g.items()}
    return loss, pack(arch, grads)


def adam_step(theta, grad, m, v, step: int, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; step counts from 1."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
