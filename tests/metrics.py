"""Error metrics against the oracle.

* E_norm,k = ||yhat_k - y_k||_2 / ||y_k||_2 over points (relative error per species);
* significant species: ||W_k w_k||_2 >= 1e-6 max_j ||W_j w_j||_2;
* E_turn,k = max_p |yhat - y| / (|y| + S_{p,k}) with the gross turnover
  S_k = sum_i |dnu_ki| (|q_f,i| + |q_r,i|) (bounded under cancellation);
* Jacobian: max_p max_j |dJ_{p,kj}| x_{p,j} / scale_{p,k} with x = (T, Y), where the row
  scale is the larger of the gross turnover S_{p,k} + |w_{p,k}| and the row's largest
  scaled entry max_j |J_{p,kj}| x_{p,j} (the T column carries the Arrhenius factor
  b + theta/T, up to ~100, that the turnover does not); row 0 (hrr) uses
  sum_k |h_k| (S_k + |w_k|) in place of the turnover.
"""
import numpy as np


def e_norm(yhat, y):
    """Per-column relative L2 error; yhat, y [n, K]."""
    num = np.sqrt(((yhat - y) ** 2).sum(axis=0))
    den = np.sqrt((y ** 2).sum(axis=0))
    return num / np.where(den > 0, den, 1.0)


def significant_species(wdot, W):
    s = np.sqrt(((wdot * W[None, :]) ** 2).sum(axis=0))
    return s >= 1e-6 * s.max()


def e_turn(yhat, y, turnover):
    return (np.abs(yhat - y) / (np.abs(y) + turnover + 1e-300)).max(axis=0)


def jac_scaled_error(Jhat, J, T, Y, turnover, wdot, h=None, hrr=None):
    """Per-row max scaled error [Ns+1] (row 0 = hrr)."""
    x = np.concatenate([np.asarray(T)[:, None], np.asarray(Y)], axis=1)          # [n, Ns+1]
    err = np.abs(Jhat - J) * x[:, None, :]                                         # [n, r, c]
    scale = np.zeros(J.shape[:2])
    scale[:, 1:] = turnover + np.abs(wdot)
    if h is not None:
        scale[:, 0] = (np.abs(h) * (turnover + np.abs(wdot))).sum(axis=1)
    else:
        scale[:, 0] = np.abs(J[:, 0, :] * x).max(axis=1)
    scale = np.maximum(scale, (np.abs(J) * x[:, None, :]).max(axis=2))
    return (err.max(axis=2) / (scale + 1e-300)).max(axis=0)
