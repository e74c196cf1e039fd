"""Fitting of the potential (Sec. II.B: the objective of eq. 7 minimized by
the BFGS method) -- oracle side.

Test infrastructure only (see ``oracle/__init__.py``).

``bfgs`` is the textbook quasi-Newton method on the inverse Hessian (the
paper cites Fletcher's book for it), written for any fun(x) -> (f, grad):

    H_0 = I; at each iterate: d = -H g; a step t is accepted when
    f(x + t d) <= f(x) + c1 t g.d (Armijo, c1 = 1e-4), halving t from t_0;
    s = t d, y = g_new - g; if y.s > 0 the inverse Hessian becomes
    H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T with rho = 1 / y.s;
    stop when max |g| <= gtol, after max_iter iterations, or when 40 halvings
    find no decrease.

Readings (the paper names the method only): an optional diagonal scale D
of the parameters (their typical sizes) gives H_0 = diag(D^2) -- the same
iterates as BFGS with H_0 = I on the parameters divided by D; before the
first update H is rescaled by y.s / y.H.y (the usual choice of the initial
inverse Hessian, (y.s / y.y) I when D = 1); the first trial step is
t_0 = min(1, 0.1 / max|D g|), so that no parameter moves by more than 0.1 D
on the first iteration; later ones start at t_0 = 1.

``fit`` applies it to eq. 7 through ``oracle.mtp.loss_and_grad``.
"""
from __future__ import annotations

import numpy as np

from . import mtp as om


def bfgs(fun, x0, max_iter, gtol=1e-10, c1=1e-4, max_halvings=40, scale=None):
    """Returns (x, f history [f(x_0), f(x_1), ...])."""
    x = np.array(x0, dtype=np.float64, copy=True)
    n = len(x)
    D = np.ones(n) if scale is None else np.asarray(scale, dtype=np.float64)
    f, g = fun(x)
    hist = [f]
    H = np.diag(D * D)
    first = True
    for _ in range(max_iter):
        if np.abs(g).max() <= gtol:
            break
        d = -H @ g
        slope = float(g @ d)
        t = min(1.0, 0.1 / np.abs(D * g).max()) if first else 1.0
        for _h in range(max_halvings):
            xn = x + t * d
            fn, gn = fun(xn)
            if fn <= f + c1 * t * slope:
                break
            t *= 0.5
        else:
            break
        s, y = xn - x, gn - g
        ys = float(y @ s)
        if ys > 0:
            if first:
                H = (ys / float(y @ H @ y)) * H
            rho = 1.0 / ys
            V = np.eye(n) - rho * np.outer(s, y)
            H = V @ H @ V.T + rho * np.outer(s, s)
            first = False
        x, f, g = xn, fn, gn
        hist.append(f)
    return x, hist


def fit(pot, theta0, configs, targets, w_e, w_f, w_s, max_iter, gtol=1e-10, scale=None):
    """BFGS on the objective of eq. 7 (configs / targets as in
    oracle.mtp.loss_and_grad).  Returns (theta, loss history)."""
    return bfgs(lambda th: om.loss_and_grad(pot, th, configs, targets, w_e, w_f, w_s), theta0, max_iter, gtol,
                scale=scale)
