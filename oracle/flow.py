"""Rational-quadratic spline coupling flow: plain FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP library and never imports it.

The learned importance sampler of the paper (section 2.3, adaptive sampling)
is a normalizing flow built from rational-quadratic spline transformations
(Durkan, Bekasov, Murray, Papamakarios 2019).  The single-bin special case of
the same spline is the RQF of the FastRambo mapping (section 2.2.9: the
equations for G_RQF, g_RQF and the closed-form inverse); that case pins the
spline formulas here.  Everything the paper leaves open (bin count, minimal
bin sizes, the derivative parametrisation, masks, network shape, loss,
optimiser) follows these readings:

* K bins on [0, 1] per transformed coordinate; widths and heights are
  ``MIN_W + (1 - K MIN_W) softmax(theta)``; the K + 1 knot derivatives are
  ``MIN_D + softplus(theta + s0)`` with ``s0 = log(exp(1 - MIN_D) - 1)`` so
  that theta = 0 gives derivative 1; knots are the cumulative sums with the
  last one set to exactly 1.  With all theta = 0 the spline is the identity.
* Coupling layer l transforms one half of the d coordinates, conditioned on
  the other half: l mod 4 = 0: the first d/2, 1: the last d/2, 2: the even
  ones, 3: the odd ones.
* The conditioner is an MLP  d/2 -> H -> H -> H -> (d/2)(3K + 1)  with ReLU
  after each hidden layer; output column ``j (3K + 1) + q`` is parameter q of
  transformed coordinate j (q < K widths, q < 2K heights, rest derivatives).
* Parameters of one layer, flat and in this order: W1 [H][d/2], b1 [H],
  W2 [H][H], b2 [H], W3 [H][H], b3 [H], W4 [(d/2)(3K+1)][H], b4; layers follow
  one another.
* Loss on a batch drawn from the flow at parameters theta_old:
  L(theta) = mean_i F_i / (q_theta(y_i) q_old,i) with F_i = (f J)^2 of the
  event, whose gradient at theta = theta_old is that of the weight variance.
* Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias correction.

Optionally the MLP is evaluated with BF16 rounding of its inputs, weights and
hidden activations (round to nearest even; accumulation, biases and the spline
in FP64), the precision model of the BF16 matrix-core kernels.
"""
from __future__ import annotations

import math

import torch

MIN_W = 1e-3
MIN_H = 1e-3
MIN_D = 1e-3
DT = torch.float64


# --------------------------------------------------------------------------
# The spline on explicit knots
# --------------------------------------------------------------------------

def rqs_bins(theta: torch.Tensor, K: int):
    """Knots (xk, yk) and knot derivatives d of the spline from its 3K + 1
    unconstrained parameters (last axis).  Shapes [..., K + 1]."""
    tw, th, td = theta[..., :K], theta[..., K:2 * K], theta[..., 2 * K:3 * K + 1]
    w = MIN_W + (1.0 - K * MIN_W) * torch.softmax(tw, dim=-1)
    h = MIN_H + (1.0 - K * MIN_H) * torch.softmax(th, dim=-1)
    s0 = math.log(math.expm1(1.0 - MIN_D))
    d = MIN_D + torch.nn.functional.softplus(td + s0)
    zero = torch.zeros(theta.shape[:-1] + (1,), dtype=theta.dtype)
    xk = torch.cat([zero, torch.cumsum(w, dim=-1)], dim=-1)
    yk = torch.cat([zero, torch.cumsum(h, dim=-1)], dim=-1)
    # the last knot is exactly 1 (cumulative sums of the widths only round to it)
    xk = torch.cat([xk[..., :K], torch.ones_like(zero)], dim=-1)
    yk = torch.cat([yk[..., :K], torch.ones_like(zero)], dim=-1)
    return xk, yk, d


def _bin(v, knots):
    """Index k of the bin [knots_k, knots_{k+1}) holding v (clamped to the
    first / last bin)."""
    K = knots.shape[-1] - 1
    k = (v.unsqueeze(-1) >= knots[..., 1:K]).sum(dim=-1)
    return k


def _take(t, k):
    return torch.gather(t, -1, k.unsqueeze(-1)).squeeze(-1)


def rqs_forward(x, xk, yk, d):
    """Monotone rational-quadratic spline x -> y on the given knots (Durkan et
    al., eqs. 4 and 5).  Returns (y, dy/dx)."""
    k = _bin(x, xk)
    x0, x1 = _take(xk, k), _take(xk, k + 1)
    y0, y1 = _take(yk, k), _take(yk, k + 1)
    d0, d1 = _take(d, k), _take(d, k + 1)
    w, h = x1 - x0, y1 - y0
    s = h / w
    xi = (x - x0) / w
    om = xi * (1.0 - xi)
    den = s + (d1 + d0 - 2.0 * s) * om
    y = y0 + h * (s * xi * xi + d0 * om) / den
    dydx = s * s * (d1 * xi * xi + 2.0 * s * om + d0 * (1.0 - xi) ** 2) / (den * den)
    return y, dydx


def rqs_inverse(y, xk, yk, d):
    """Inverse of rqs_forward: the root in [0, 1] of the quadratic for the bin
    coordinate, in the cancellation-free form 2c / (-b - sqrt(b^2 - 4ac)).
    Returns (x, dx/dy)."""
    k = _bin(y, yk)
    x0, x1 = _take(xk, k), _take(xk, k + 1)
    y0, y1 = _take(yk, k), _take(yk, k + 1)
    d0, d1 = _take(d, k), _take(d, k + 1)
    w, h = x1 - x0, y1 - y0
    s = h / w
    dy = y - y0
    kap = d1 + d0 - 2.0 * s
    a = h * (s - d0) + dy * kap
    b = h * d0 - dy * kap
    c = -s * dy
    disc = torch.clamp(b * b - 4.0 * a * c, min=0.0)
    xi = 2.0 * c / (-b - torch.sqrt(disc))
    x = x0 + xi * w
    om = xi * (1.0 - xi)
    den = s + kap * om
    dydx = s * s * (d1 * xi * xi + 2.0 * s * om + d0 * (1.0 - xi) ** 2) / (den * den)
    return x, 1.0 / dydx


# --------------------------------------------------------------------------
# Coupling flow
# --------------------------------------------------------------------------

def bf16(t: torch.Tensor) -> torch.Tensor:
    """Round to the nearest BF16 value (ties to even), returned in FP64.
    Gradients pass straight through."""
    # through FP32, as the kernels round their FP32 values
    r = t.detach().to(torch.float32).to(torch.bfloat16).to(DT)
    return t + (r - t).detach()


def transformed(d: int, layer: int):
    """Indices of the coordinates coupling layer `layer` transforms."""
    m = layer % 4
    if m == 0:
        return list(range(d // 2))
    if m == 1:
        return list(range(d // 2, d))
    if m == 2:
        return list(range(0, d, 2))
    return list(range(1, d, 2))


def conditioning(d: int, layer: int):
    t = set(transformed(d, layer))
    return [i for i in range(d) if i not in t]


class Flow:
    """Coupling flow with flat FP64 parameters (see the module docstring for
    the layout)."""

    def __init__(self, dims: int, layers: int = 8, bins: int = 16, hidden: int = 128, params=None,
                 bf16_mlp: bool = False):
        if dims % 2:
            raise ValueError("dims must be even")
        self.d, self.L, self.K, self.H = dims, layers, bins, hidden
        self.bf16 = bf16_mlp
        self.n_half = dims // 2
        self.n_out = self.n_half * (3 * bins + 1)
        self.shapes = [(hidden, self.n_half), (hidden,), (hidden, hidden), (hidden,), (hidden, hidden), (hidden,),
                       (self.n_out, hidden), (self.n_out,)]
        self.per_layer = sum(math.prod(s) for s in self.shapes)
        self.n_params = self.per_layer * layers
        p = torch.zeros(self.n_params, dtype=DT) if params is None else torch.as_tensor(params, dtype=DT).clone()
        if p.numel() != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {p.numel()}")
        self.params = p

    def layer_tensors(self, params, layer):
        off = layer * self.per_layer
        out = []
        for s in self.shapes:
            n = math.prod(s)
            out.append(params[off:off + n].reshape(s))
            off += n
        return out

    def mlp(self, params, layer, cond):
        """Spline parameters [n, d/2, 3K+1] from the conditioning coordinates
        [n, d/2]."""
        W1, b1, W2, b2, W3, b3, W4, b4 = self.layer_tensors(params, layer)
        r = bf16 if self.bf16 else (lambda t: t)
        h = r(cond)
        h = r(torch.relu(h @ r(W1).T + b1))
        h = r(torch.relu(h @ r(W2).T + b2))
        h = r(torch.relu(h @ r(W3).T + b3))
        out = h @ r(W4).T + b4
        return out.reshape(-1, self.n_half, 3 * self.K + 1)

    def forward(self, u, params=None):
        """u [n, d] in (0,1)^d -> (y [n, d], log|dy/du| [n])."""
        params = self.params if params is None else params
        z = torch.as_tensor(u, dtype=DT).clone()
        logdet = torch.zeros(z.shape[0], dtype=DT)
        for layer in range(self.L):
            t, c = transformed(self.d, layer), conditioning(self.d, layer)
            theta = self.mlp(params, layer, z[:, c])
            xk, yk, dk = rqs_bins(theta, self.K)
            y, dydx = rqs_forward(z[:, t], xk, yk, dk)
            z = z.clone()
            z[:, t] = y
            logdet = logdet + torch.log(dydx).sum(dim=1)
        return z, logdet

    def inverse(self, y, params=None):
        """y [n, d] -> (u [n, d], log|du/dy| [n]); log q(y) is the second."""
        params = self.params if params is None else params
        z = torch.as_tensor(y, dtype=DT).clone()
        logdet = torch.zeros(z.shape[0], dtype=DT)
        for layer in reversed(range(self.L)):
            t, c = transformed(self.d, layer), conditioning(self.d, layer)
            theta = self.mlp(params, layer, z[:, c])
            xk, yk, dk = rqs_bins(theta, self.K)
            x, dxdy = rqs_inverse(z[:, t], xk, yk, dk)
            z = z.clone()
            z[:, t] = x
            logdet = logdet + torch.log(dxdy).sum(dim=1)
        return z, logdet

    def loss(self, y, F, logq_old, params=None):
        """Variance loss mean(F / (q_theta(y) q_old)) of a batch."""
        _, logq = self.inverse(y, params)
        F = torch.as_tensor(F, dtype=DT)
        lqo = torch.as_tensor(logq_old, dtype=DT)
        return torch.mean(F * torch.exp(-logq - lqo))

    def loss_and_grad(self, y, F, logq_old):
        """Loss and its gradient with respect to the flat parameters (reverse
        mode through the inverse pass)."""
        p = self.params.clone().requires_grad_(True)
        L = self.loss(y, F, logq_old, p)
        (g,) = torch.autograd.grad(L, p)
        return float(L.detach()), g.detach()


class Adam:
    """Adam with bias correction (Kingma and Ba 2015)."""

    def __init__(self, n, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.m = torch.zeros(n, dtype=DT)
        self.v = torch.zeros(n, dtype=DT)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, params, grad):
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * grad
        self.v = self.b2 * self.v + (1.0 - self.b2) * grad * grad
        mh = self.m / (1.0 - self.b1 ** self.t)
        vh = self.v / (1.0 - self.b2 ** self.t)
        return params - self.lr * mh / (torch.sqrt(vh) + self.eps)
