"""Error metrics against the oracle.

* E_norm,k = ||yhat_k - y_k||_2 / ||y_k||_2 over points (relative error per species);
* significant species: ||W_k w_k||_2 >= 1e-6 max_j ||W_j w_j||_2;
* E_turn,k = max_p |yhat - y| / (|y| + S_{p,k}) with the gross turnover
  S_k = sum_i |dnu_ki| (|q_f,i| + |q_r,i|) (bounded under cancellation);
* Jacobian: with x = (T, Y) and G the gross Jacobian of the oracle (every reaction's
  chain-rule terms in absolute value), the T column of row k is measured against its own
  gross value, |dJ_{p,k0}| / G_{p,k0}, and the Y columns against the largest gross Y entry
  of the row, |dJ_{p,kj}| Y_j / max_{j>=1} G_{p,kj} Y_j: G bounds the rounding of any
  summation order, as the gross turnover does for w (entries of J cancel across
  reactions), and the T column, which carries the Arrhenius factor b + theta/T, never
  sets the scale of the Y columns;
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


def jac_scaled_errors(Jhat, J, G, T, Y, floor=0.0):
    """Per-row max scaled error of the T column and of the Y columns, each [Ns+1] (row 0 = hrr).

    T column: |dJ_k0| T / (G_k0 T); Y columns: max_j |dJ_kj| Y_j / max_j (G_kj Y_j).
    floor > 0 measures a row whose scale is below floor x the point's largest scale of the
    same column group against that floor instead: an FP32 Jacobian cannot hold rows that
    are, say, 1e-60 of the point's dominant rows (they flush to zero), and such rows carry
    no weight in a Newton iteration.
    """
    T = np.asarray(T)
    Y = np.asarray(Y)
    dJ = np.abs(Jhat - J)
    errT = dJ[:, :, 0]                                                     # [n, r]
    scT = G[:, :, 0]
    errY = (dJ[:, :, 1:] * Y[:, None, :]).max(axis=2)
    scY = (G[:, :, 1:] * Y[:, None, :]).max(axis=2)
    if floor > 0:
        scT = np.maximum(scT, floor * scT.max(axis=1, keepdims=True))
        scY = np.maximum(scY, floor * scY.max(axis=1, keepdims=True))
    return (errT / (scT + 1e-300)).max(axis=0), (errY / (scY + 1e-300)).max(axis=0)


def jac_scaled_error(Jhat, J, G, T, Y, floor=0.0):
    """Per-row max of the T-column and Y-column scaled errors (jac_scaled_errors), [Ns+1]."""
    eT, eY = jac_scaled_errors(Jhat, J, G, T, Y, floor=floor)
    return np.maximum(eT, eY)


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
