"""Parity measures between the HIP path and the CPU oracle.

Image: a pixel is a branch flip if any channel differs by more than
1e-3 * max(|I_oracle|, mean |I_oracle|); no pixel may flip (both sides take
every discrete decision on the same binary32 values, so a flip is a mistake on
one side, not rounding), and the relative RMSE over all pixels must be
<= 1e-4 (the pixel means differ in the last bits only: the oracle adds a
pixel's samples in binary64, the HIP path in binary32 in sample order).
Gradient: |g_gpu - g_oracle| <= 1e-4 * S_j per component, with
S_j = (1/P) sum_p |c_pj| (L_2p + L_2p+1), the scale of the terms whose
difference the estimator takes.  Per-image loss: relative error <= 1e-4.
"""
import numpy as np

FLIP_FRAC = 0.0
REL_RMSE = 1e-4
GRAD_REL = 1e-4
LOSS_REL = 1e-4


def image_stats(gpu, orc):
    g = np.asarray(gpu, np.float64).reshape(-1, 3)
    o = np.asarray(orc, np.float64).reshape(-1, 3)
    mean = np.abs(o).mean()
    thr = 1e-3 * np.maximum(np.abs(o), mean)
    flip = (np.abs(g - o) > thr).any(axis=1)
    keep = ~flip
    den = np.linalg.norm(o)
    num = np.linalg.norm((g - o)[keep])
    rel = num / den if den > 0 else num
    return dict(flip_frac=float(flip.mean()), flips=int(flip.sum()), rel_rmse=float(rel),
                max_abs=float(np.abs(g - o).max()) if g.size else 0.0)


def assert_images_match(gpu, orc, what=""):
    st = image_stats(gpu, orc)
    assert st["flip_frac"] <= FLIP_FRAC, (what, st)
    assert st["rel_rmse"] <= REL_RMSE, (what, st)
    return st


def grad_scale(c, L):
    """S_j = (1/P) sum_p |c_pj| (L_2p + L_2p+1) for antithetic pair weights, or
    (1/N) sum_i |c_ij| L_i for independent draws (one weight row per loss)."""
    c = np.asarray(c, np.float64)
    L = np.asarray(L, np.float64)
    if c.shape[0] == L.shape[0]:
        return (np.abs(c) * L[:, None]).mean(axis=0)
    return (np.abs(c) * (L[0::2] + L[1::2])[:, None]).mean(axis=0)


def assert_grad_match(g_gpu, g_orc, c, L_orc, what=""):
    S = grad_scale(c, L_orc)
    err = np.abs(np.asarray(g_gpu) - np.asarray(g_orc))
    assert np.all(err <= GRAD_REL * S + 1e-300), (what, err, S, g_gpu, g_orc)
    return err / np.maximum(S, 1e-300)


def assert_losses_match(L_gpu, L_orc, what=""):
    L_gpu, L_orc = np.asarray(L_gpu), np.asarray(L_orc)
    rel = np.abs(L_gpu - L_orc) / np.maximum(np.abs(L_orc), 1e-300)
    assert np.all(rel <= LOSS_REL), (what, rel)
    return rel
