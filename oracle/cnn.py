"""Small convolutional score network: forward, hand-written backward, Adam; FP64.

Test infrastructure (see ``oracle/__init__``).

The paper closes by proposing learned score functions for AMS (Conclusion).
The network used for that here is fixed by the workload: three 3x3
convolutions with 32 output channels (zero padding 1, stride 1, ReLU after
each), a global average over the 16x16 positions and a linear read-out to one
number.  Layout NCHW; weights [C_out, C_in, 3, 3].  A convolution is the
cross-correlation
    Z[b, o, y, x] = bias[o] + sum_{c, dy, dx} W[o, c, dy, dx] Xp[b, c, y + dy, x + dx]
with Xp the input padded by one zero row/column on every side.

Loss: mean squared error (1/B) sum_b (y_b - label_b)^2.  Adam (Kingma & Ba,
2015) with bias correction updates FP64 master weights.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Dict, Optional

import numpy as np

CH = 32
H = 16
NAMES = ("w1", "b1", "w2", "b2", "w3", "b3", "w4", "b4")


def shapes(c_in: int = 3) -> Dict[str, tuple]:
    return {"w1": (CH, c_in, 3, 3), "b1": (CH,), "w2": (CH, CH, 3, 3), "b2": (CH,),
            "w3": (CH, CH, 3, 3), "b3": (CH,), "w4": (CH,), "b4": ()}


def pad1(x: np.ndarray) -> np.ndarray:
    return np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Zero-padded 3x3 cross-correlation, [B, C, H, W] -> [B, O, H, W]."""
    xp = pad1(x)
    bsz, _, hh, ww = x.shape
    out = np.zeros((bsz, w.shape[0], hh, ww))
    for dy in range(3):
        for dx in range(3):
            out += np.einsum("oc,bcyx->boyx", w[:, :, dy, dx], xp[:, :, dy:dy + hh, dx:dx + ww])
    return out + b[None, :, None, None]


def conv3x3_input_grad(gz: np.ndarray, w: np.ndarray) -> np.ndarray:
    """d loss / d x for Z = conv3x3(x, w, b): each output tap sends its gradient back."""
    bsz, _, hh, ww = gz.shape
    gxp = np.zeros((bsz, w.shape[1], hh + 2, ww + 2))
    for dy in range(3):
        for dx in range(3):
            gxp[:, :, dy:dy + hh, dx:dx + ww] += np.einsum("oc,boyx->bcyx", w[:, :, dy, dx], gz)
    return gxp[:, :, 1:-1, 1:-1]


def conv3x3_weight_grad(gz: np.ndarray, x: np.ndarray) -> np.ndarray:
    """d loss / d W for Z = conv3x3(x, w, b)."""
    xp = pad1(x)
    _, _, hh, ww = x.shape
    gw = np.zeros((gz.shape[1], x.shape[1], 3, 3))
    for dy in range(3):
        for dx in range(3):
            gw[:, :, dy, dx] = np.einsum("boyx,bcyx->oc", gz, xp[:, :, dy:dy + hh, dx:dx + ww])
    return gw


def forward(p: Dict[str, np.ndarray], x: np.ndarray, layer_input: Optional[Callable] = None):
    """Returns (y [B], cache) for inputs x [B, C, 16, 16].

    layer_input, if given, is applied to the input of each convolution (x, and
    the activations of the first two layers) before it is convolved: a network
    whose matrix products take their inputs in a narrower format (BF16) is this
    one with the rounding to that format as layer_input.  The cache holds the
    layer inputs as convolved, so the backward pass takes the rounding's
    derivative as 1 (the weight gradients use the inputs the products saw)."""
    li = (lambda a: a) if layer_input is None else layer_input
    x_in = li(x)
    z1 = conv3x3(x_in, p["w1"], p["b1"])
    a1 = li(np.maximum(z1, 0.0))
    z2 = conv3x3(a1, p["w2"], p["b2"])
    a2 = li(np.maximum(z2, 0.0))
    z3 = conv3x3(a2, p["w3"], p["b3"])
    a3 = np.maximum(z3, 0.0)
    g = a3.mean(axis=(2, 3))
    y = g @ p["w4"] + p["b4"]
    return y, dict(x=x_in, z1=z1, a1=a1, z2=z2, a2=a2, z3=z3, a3=a3, g=g)


def loss(y: np.ndarray, label: np.ndarray) -> float:
    return float(np.mean((y - label) ** 2))


def backward(p: Dict[str, np.ndarray], cache, y: np.ndarray, label: np.ndarray) -> Dict[str, np.ndarray]:
    """Gradients of the MSE loss with respect to every parameter."""
    bsz = y.shape[0]
    gy = 2.0 * (y - label) / bsz
    grads = {"w4": cache["g"].T @ gy, "b4": np.array(gy.sum())}
    gg = np.outer(gy, p["w4"])
    hw = cache["a3"].shape[2] * cache["a3"].shape[3]
    ga3 = np.broadcast_to(gg[:, :, None, None] / hw, cache["a3"].shape)
    gz3 = ga3 * (cache["z3"] > 0)
    grads["w3"] = conv3x3_weight_grad(gz3, cache["a2"])
    grads["b3"] = gz3.sum(axis=(0, 2, 3))
    ga2 = conv3x3_input_grad(gz3, p["w3"])
    gz2 = ga2 * (cache["z2"] > 0)
    grads["w2"] = conv3x3_weight_grad(gz2, cache["a1"])
    grads["b2"] = gz2.sum(axis=(0, 2, 3))
    ga1 = conv3x3_input_grad(gz2, p["w2"])
    gz1 = ga1 * (cache["z1"] > 0)
    grads["w1"] = conv3x3_weight_grad(gz1, cache["x"])
    grads["b1"] = gz1.sum(axis=(0, 2, 3))
    return grads


@dataclass
class Adam:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    t: int = 0
    m: Dict[str, np.ndarray] = field(default_factory=dict)
    v: Dict[str, np.ndarray] = field(default_factory=dict)

    def step(self, p: Dict[str, np.ndarray], g: Dict[str, np.ndarray]) -> None:
        self.t += 1
        for name in NAMES:
            if name not in self.m:
                self.m[name] = np.zeros_like(p[name])
                self.v[name] = np.zeros_like(p[name])
            self.m[name] = self.beta1 * self.m[name] + (1 - self.beta1) * g[name]
            self.v[name] = self.beta2 * self.v[name] + (1 - self.beta2) * g[name] ** 2
            mhat = self.m[name] / (1 - self.beta1 ** self.t)
            vhat = self.v[name] / (1 - self.beta2 ** self.t)
            p[name] = p[name] - self.lr * mhat / (np.sqrt(vhat) + self.eps)
