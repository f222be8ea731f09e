"""Learned per-point weights that precondition the least-squares inverse.

The paper runs its transforms inside iterative inverse algorithms (Sec. I) but proposes no
preconditioner; this module is an extension built on the library's own kernels:

* ``LearnedWeights.features``: a coarse density map of the point set and 12 features per
  point (``nusht_density_map``, ``nusht_point_features``);
* ``LearnedWeights.weights``: w_i = softplus(net(features_i)) * 4 pi / N from a
  12 -> 128 -> 128 -> 128 -> 1 FP32 network (``nusht_mlp_forward``);
* ``LearnedWeights.train``: Adam on L(w) = sum over training sets of
  <r, r>_m / <a*, a*>_m, r = S^H (W d) - a*.  Its gradient with respect to w costs one
  adjoint and one synthesis (``nusht_weight_loss_grad``) and flows back through the network
  (``nusht_mlp_backward``, ``nusht_adam_step``);
* ``solve_weighted``: CGLS on W^(1/2) S from x0 = S^H W d (``nusht_solve``), with plain
  CGLS from zero as the fallback.

This file only marshals arguments; every numeric step runs in the library.  The network's
initial parameters are a seeded random draw made here on the host.
"""
from __future__ import annotations

import math

import numpy as np

from . import _binding as B

SIZES = (12, 128, 128, 128, 1)


def init_params(seed: int = 0) -> np.ndarray:
    """Flat FP32 parameters in the library's layout (per layer: transposed weight [in][out],
    then bias).  Hidden weights ~ N(0, 1 / fan_in); the output layer starts small with bias
    log(e - 1) so that every initial weight is close to softplus(log(e - 1)) * scale = scale,
    i.e. the plain equal-area quadrature 4 pi / N."""
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(len(SIZES) - 1):
        nin, nout = SIZES[i], SIZES[i + 1]
        W = rng.standard_normal((nin, nout)) / math.sqrt(nin)
        b = np.zeros(nout)
        if i == len(SIZES) - 2:
            W *= 0.1
            b[:] = math.log(math.e - 1.0)
        parts += [W.ravel(), b]
    flat = np.concatenate(parts).astype(np.float32)
    assert flat.size == B.mlp_param_count()
    return flat


class LearnedWeights:
    """The network's parameters (a float32 device tensor) plus the density-map size."""

    def __init__(self, ntheta: int = 64, nphi: int = 128, seed: int = 0, params=None,
                 device="cuda"):
        import torch
        self.ntheta, self.nphi = int(ntheta), int(nphi)
        if params is None:
            params = init_params(seed)
        self.params = torch.as_tensor(np.asarray(params, dtype=np.float32)).to(device).contiguous()
        self.step = 0
        self._m = torch.zeros_like(self.params)
        self._v = torch.zeros_like(self.params)

    # ---- inference ----
    def features(self, theta, phi):
        rho = B.density_map(theta, phi, self.ntheta, self.nphi)
        return B.point_features(theta, phi, rho)

    @staticmethod
    def scale(npts: int) -> float:
        return 4.0 * math.pi / npts

    def weights(self, theta=None, phi=None, features=None):
        if features is None:
            features = self.features(theta, phi)
        return B.mlp_forward(self.params, features, self.scale(features.shape[0]))

    # ---- training ----
    def train(self, examples, steps: int, lr: float = 1e-3, log=None):
        """examples: list of dicts with 'plan' (a Plan), 'features' [N, 12] float32, 'd' [N]
        float64 and 'astar' [nalm] complex128, all on the device and with the same N.  Each
        step sums the loss over the examples and takes one Adam step.  Returns the per-step
        summed losses."""
        import torch
        n = {int(e["features"].shape[0]) for e in examples}
        if len(n) != 1:
            raise ValueError("training sets must have the same number of points")
        npts = n.pop()
        feats = torch.cat([e["features"] for e in examples]).contiguous()
        hist = []
        for _ in range(steps):
            w = B.mlp_forward(self.params, feats, self.scale(npts))
            gws = []
            total = 0.0
            for k, e in enumerate(examples):
                loss, g = e["plan"].weight_loss_grad(e["d"], e["astar"],
                                                      w[k * npts:(k + 1) * npts])
                total += loss
                gws.append(g)
            grad = B.mlp_backward(self.params, feats, torch.cat(gws), self.scale(npts))
            self.step += 1
            B.adam_step(self.params, grad, self._m, self._v, self.step, lr=lr)
            hist.append(total)
            if log is not None:
                log(self.step, total)
        return hist

    # ---- persistence ----
    def state(self) -> dict:
        return dict(params=self.params.cpu().numpy(), m=self._m.cpu().numpy(),
                    v=self._v.cpu().numpy(), step=self.step, ntheta=self.ntheta,
                    nphi=self.nphi)

    def save(self, path: str):
        np.savez(path, **self.state())

    @classmethod
    def load(cls, path: str, device="cuda"):
        import torch
        z = np.load(path)
        lw = cls(int(z["ntheta"]), int(z["nphi"]), params=z["params"], device=device)
        lw._m = torch.as_tensor(z["m"]).to(device).contiguous()
        lw._v = torch.as_tensor(z["v"]).to(device).contiguous()
        lw.step = int(z["step"])
        return lw


def solve_weighted(plan, d, weights, tol=1e-8, maxiter=1000, fallback=True):
    """CGLS on W^(1/2) S started from x0 = S^H W d (``nusht_weighted_adjoint``,
    ``nusht_solve``).  If that does not converge within maxiter and ``fallback`` is set, plain
    CGLS from zero is run instead.  Returns (alm, iterations, true relative residual, status,
    used_fallback); iterations include the failed weighted attempt."""
    x0 = plan.weighted_adjoint(d, weights)
    x, it, rr, st = plan.solve(d, x0=x0, weights=weights, tol=tol, maxiter=maxiter, check=False)
    if st == B.NUSHT_OK or not fallback:
        return x, it, rr, st, False
    x2, it2, rr2, st2 = plan.solve(d, tol=tol, maxiter=maxiter, check=False)
    return x2, it + it2, rr2, st2, True
