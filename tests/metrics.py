"""Error metrics against the oracle.

* E_norm,k = ||yhat_k - y_k||_2 / ||y_k||_2 over points (relative error per species);
* significant species: ||W_k w_k||_2 >= 1e-6 max_j ||W_j w_j||_2;
* E_turn,k = max_p |yhat - y| / (|y| + S_{p,k}) with the gross turnover
  S_k = sum_i |dnu_ki| (|q_f,i| + |q_r,i|) (bounded under cancellation);
* Jacobian: max_p max_j |dJ_{p,kj}| x_{p,j} / max_j (G_{p,kj} x_{p,j}) with x = (T, Y) and G
  the gross Jacobian of the oracle (every reaction's chain-rule terms in absolute value):
  the row scale bounds the rounding of any summation order, as the gross turnover does
  for w (entries of J cancel across reactions, and the T column carries the Arrhenius
  factor b + theta/T that the turnover alone does not);
* VJP: |dg_x| / sum_r |u_r| G_rx.
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


def jac_scaled_error(Jhat, J, G, T, Y, floor=0.0):
    """Per-row max scaled error [Ns+1] (row 0 = hrr); G is the oracle's gross Jacobian.

    floor > 0 measures rows whose gross scale is below floor x the point's largest row
    scale against that floor instead: an FP32 Jacobian cannot hold rows that are, say,
    1e-60 of the point's dominant rows (they flush to zero), and such rows carry no
    weight in a Newton iteration.
    """
    x = np.concatenate([np.asarray(T)[:, None], np.asarray(Y)], axis=1)          # [n, Ns+1]
    err = np.abs(Jhat - J) * x[:, None, :]                                         # [n, r, c]
    scale = (G * x[:, None, :]).max(axis=2)
    if floor > 0:
        scale = np.maximum(scale, floor * scale.max(axis=1, keepdims=True))
    return (err.max(axis=2) / (scale + 1e-300)).max(axis=0)


FLT_MAX = float(np.finfo(np.float32).max)


def fp32_range_split(Jhat, J):
    """(Jhat', J') with entries whose exact value exceeds the FP32 range removed, after
    checking that the FP32 result holds an infinity of the right sign there."""
    big = np.abs(J) > FLT_MAX
    assert np.all(np.isinf(Jhat[big]) & (np.sign(Jhat[big]) == np.sign(J[big])))
    return np.where(big, 0.0, Jhat), np.where(big, 0.0, J)


def vjp_scaled_error(g_hat, g_ref, u_full, G):
    """max |g_hat - g_ref| / sum_r |u_r| G_rc; u_full [n, Ns+1] includes the hrr cotangent."""
    scale = np.einsum("nr,nrc->nc", np.abs(u_full), G) + 1e-300
    return np.max(np.abs(g_hat - g_ref) / scale)
