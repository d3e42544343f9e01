"""Surrogate-bracketed critical-pressure solves.

The critical forcing of a channel problem is found by the library's batched
bisection (lbm_critical_pressure).  A plain solve bisects over a bracket of
three decades of Bond number; a surrogate solve starts from a narrow bracket
proposed by the network of include/lbm_mlp.h, trained on the results of
earlier solves, and lets the driver check lazily that the converged bracket
really contains the threshold (verify_bracket = 2), widening it when the
proposal was wrong.  The simulation therefore always decides the result;
the network only saves probes.

Features of a problem (the inputs of the network):
    [log2 lambda, h0 / lambda, a / lambda, cos theta, log10 M, L_slug / lambda]
with M = nu_o / nu_w = (tau_o - 1/2) / (tau_w - 1/2); target: log10 Bo_c with
Bo = rho_bar g L D / sigma, L = nx (the channel length), D = h0 - a (Eq. 15).
Everything numeric runs in the library (HIP kernels); this module only
standardises features, batches calls and converts units.
"""
import math

import numpy as np

from . import binding, mlp


def features(cfg):
    lam = float(cfg["lam"])
    tau_o, tau_w = cfg["tau"]
    M = (tau_o - 0.5) / (tau_w - 0.5)
    return np.array([math.log2(lam), cfg["h0"] / lam, cfg["a"] / lam,
                     math.cos(math.radians(cfg["theta"])), math.log10(M),
                     cfg["init"]["length"] / lam])


def bond_scale(cfg, sigma, rho_bar):
    """Bo / g for this problem (Eq. 15 with L = nx, D = h0 - a)."""
    return rho_bar * cfg["nx"] * (cfg["h0"] - cfg["a"]) / sigma


def plain_bracket(cfg, sigma, rho_bar, decades=3.0):
    """The plain solve's bracket: Bo in 10^(-decades/2) .. 10^(decades/2)."""
    s = bond_scale(cfg, sigma, rho_bar)
    return 10.0 ** (-0.5 * decades) / s, 10.0 ** (0.5 * decades) / s


def step_rules(cfg, base_lam=64.0, equil=4000, min_steps=5000, max_steps=30000):
    """Per-problem step counts scaled from a lambda = 64 channel: relaxation
    (equilibration, the minimum before calling a probe static) grows like
    lambda^2 at fixed Bo, the travel of half a wavelength like lambda."""
    r = cfg["lam"] / base_lam
    return dict(equil_steps=int(equil * r * r), min_steps=int(min_steps * r * r),
                max_steps=int(max(max_steps * r, min_steps * r * r + 10000 * r)))


def solve(cfgs, brackets, sigma, rho_bar, rules=step_rules, stream=None, **options):
    """Batched critical-pressure solve of every problem; returns the
    library's result dicts (g_lo, g_hi, g_crit, bo_crit, probes, flags, steps).
    rules(cfg) gives equil_steps, min_steps and max_steps per problem."""
    probs = []
    for c, (lo, hi) in zip(cfgs, brackets):
        r = rules(c)
        probs.append(binding.cp_problem(c, lo, hi, sigma, rho_bar, r["equil_steps"],
                                        r["max_steps"], min_steps=r["min_steps"]))
    return binding.lbm_critical_pressure(probs, binding.cp_options(**options), stream=stream)


class Surrogate:
    """Network plus the standardisation of its inputs and target."""

    def __init__(self, init_params, max_batch=1024):
        self.net = mlp.Network(init_params, max_batch=max_batch)
        self.x_mean = self.x_std = None
        self.y_mean, self.y_std = 0.0, 1.0
        self.sigma_val = None
        self.history = []

    def _std_x(self, F):
        return ((np.asarray(F, dtype=np.float64) - self.x_mean) / self.x_std).astype(np.float32)

    def fit(self, F, log_bo, rng, epochs=400, batch=64, lr=2e-3, val_frac=0.2):
        """Train on features F [N, 6] and targets log10 Bo_c [N] with Adam on
        shuffled minibatches (rng: numpy Generator for the split and the
        shuffles); keeps the validation RMSE (log10 units) as sigma_val."""
        import torch
        F = np.asarray(F, dtype=np.float64)
        y = np.asarray(log_bo, dtype=np.float64)
        n = len(y)
        perm = rng.permutation(n)
        n_val = max(1, int(round(val_frac * n))) if n > 4 else 0
        val, tr = perm[:n_val], perm[n_val:]
        self.x_mean = F[tr].mean(axis=0)
        self.x_std = np.where(F[tr].std(axis=0) > 1e-12, F[tr].std(axis=0), 1.0)
        self.y_mean = float(y[tr].mean())
        self.y_std = float(y[tr].std()) if y[tr].std() > 1e-12 else 1.0
        X = torch.from_numpy(self._std_x(F)).cuda()
        T = torch.from_numpy(((y - self.y_mean) / self.y_std).astype(np.float32)).cuda()
        b = min(batch, len(tr), self.net.max_batch)
        for ep in range(epochs):
            order = tr[rng.permutation(len(tr))]
            for s in range(0, len(order) - b + 1, b):
                idx = torch.from_numpy(order[s:s + b]).cuda()
                self.net.train_step(X[idx].contiguous(), T[idx].contiguous(), lr=lr)
            if ep % 50 == 49 or ep == epochs - 1:
                self.history.append((ep + 1, float(self.net.loss.cpu())))
        if n_val:
            pred = self.predict(F[val])
            self.sigma_val = float(np.sqrt(np.mean((pred - y[val]) ** 2)))
        return self

    def predict(self, F):
        """Predicted log10 Bo_c for features F [N, 6]."""
        out = self.net.predict(self._std_x(np.atleast_2d(F)))
        return out.cpu().numpy().astype(np.float64) * self.y_std + self.y_mean

    def brackets(self, cfgs, sigma, rho_bar, k=2.0, floor=0.01):
        """Proposed brackets: predicted log10 Bo_c +- max(k sigma_val, floor)."""
        pred = self.predict(np.stack([features(c) for c in cfgs]))
        half = max(k * (self.sigma_val or 0.0), floor)
        out = []
        for c, p in zip(cfgs, pred):
            s = bond_scale(c, sigma, rho_bar)
            out.append((10.0 ** (p - half) / s, 10.0 ** (p + half) / s))
        return out
