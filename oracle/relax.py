"""Residual-based relaxation and the harmonic side of the FBC loop (FP64 oracle;
test infrastructure only).

Section 2.3.3, eq. alpha with v = f_in,k+1 - f_in,k (Aitken / Lemarechal), and
Algorithm 2 (Relax):
    alpha_{k+1} = -alpha_k <f_k, f_{k+1} - f_k> / ||f_{k+1} - f_k||^2
    alpha_{k+1} < 0  ->  alpha_{k+1} = 1
    optional: if ||alpha_{k+1} G f_{k+1}||_inf > du_max, alpha_{k+1} = du_max / ||G f_{k+1}||_inf
Algorithm 1, relaxation and update: relaxation only when enabled and k >= 2 (alpha = 1 before,
with alpha_2 = 1 as the starting value); the update uses alpha_{k+1} f_in,k+1 while
Relax always receives the raw (unscaled) incompatibility forces; then the pad
update and mean removal.  The incompatibility-force criterion of Section 2.3.3
(||f_in||_inf < tol) is reported as the convergence flag.

Variant (the Remark in Section 2.3.3, the preprint's choice): a lower bound alpha_min on
alpha_{k+1} in place of the incompatibility-force criterion.

Readings where the paper is silent: a zero denominator keeps alpha_{k+1} = alpha_k;
every RHS is an independent FBC iteration with its own alpha; the lower bound acts after
the reset of negative values and before the optional step bound (which stays a hard
bound on the step).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .apply import pad_update


def relax_alpha(f_new: np.ndarray, f_old: np.ndarray, alpha_old: np.ndarray,
                alpha_min: float = 0.0) -> np.ndarray:
    """Algorithm 2, the residual-based alpha (eq. alpha), per RHS (leading axis); alpha_min > 0: the lower bound of the
    Remark in Section 2.3.3."""
    n = f_new.shape[0]
    fn = f_new.reshape(n, -1)
    fo = f_old.reshape(n, -1)
    d = fn - fo
    num = np.einsum("rj,rj->r", fo, d)
    den = np.einsum("rj,rj->r", d, d)
    out = np.array(alpha_old, dtype=np.float64, copy=True)
    nz = den > 0.0
    out[nz] = -alpha_old[nz] * num[nz] / den[nz]
    out[out < 0.0] = 1.0
    if alpha_min > 0.0:
        out = np.maximum(out, alpha_min)
    return out


def clamp_step(alpha: np.ndarray, w_inf: np.ndarray, du_max: float) -> np.ndarray:
    """Algorithm 2, the optional step bound."""
    out = alpha.copy()
    hit = alpha * w_inf > du_max
    out[hit] = du_max / w_inf[hit]
    return out


@dataclass
class RelaxState:
    n_rhs: int
    relax: bool = True
    du_max: float = 0.0          # <= 0 disables the step bound
    tol_f: float = 1e-3
    alpha_min: float = 0.0       # > 0: lower bound on alpha (Remark in Section 2.3.3)
    k: int = 0
    alpha: np.ndarray = field(default=None)
    f_prev: np.ndarray = field(default=None)

    def __post_init__(self):
        if self.alpha is None:
            self.alpha = np.ones(self.n_rhs)


def relax_step(state: RelaxState, f_new: np.ndarray, u: np.ndarray, apply_fn) -> tuple[np.ndarray, dict]:
    """One pass of Algorithm 1 from the relaxation on, given f_in,k+1 (supplied by the caller).

    apply_fn(f) must return G^{p|i+} f with the layout of u.  Returns (u_new, out)."""
    n = f_new.shape[0]
    w = apply_fn(f_new)
    w_inf = np.abs(w.reshape(n, -1)).max(axis=1)
    if state.relax and state.k >= 2:
        alpha = relax_alpha(f_new, state.f_prev, state.alpha, state.alpha_min)
        if state.du_max > 0.0:
            alpha = clamp_step(alpha, w_inf, state.du_max)
    else:
        alpha = np.ones(n)
    u_new, mean = pad_update(u, w, alpha)
    f_inf = np.abs(f_new.reshape(n, -1)).max(axis=1)
    out = dict(alpha=alpha.copy(), f_inf=f_inf, step_inf=alpha * w_inf, mean_removed=mean,
               converged=(f_inf < state.tol_f))
    state.alpha = alpha
    state.f_prev = np.array(f_new, copy=True)
    state.k += 1
    return u_new, out
