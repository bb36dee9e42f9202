"""Shared helpers of the test-suite: pair data of an oracle iterate in the
stateless-batch format, and the scaled error measures the parity bar uses."""
import numpy as np

import workloads


def rotation(prob, s):
    if prob["dim"] == 2:
        th = s[prob["att_idx"][0]]
        return np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    ph, th, ps = (s[i] for i in prob["att_idx"])
    Rx = np.array([[1, 0, 0], [0, np.cos(ph), -np.sin(ph)], [0, np.sin(ph), np.cos(ph)]])
    Ry = np.array([[np.cos(th), 0, np.sin(th)], [0, 1, 0], [-np.sin(th), 0, np.cos(th)]])
    Rz = np.array([[np.cos(ps), -np.sin(ps), 0], [np.sin(ps), np.cos(ps), 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def pair_geometry(prob, state, b, t, layout=None):
    """(A, b, Cp, dp) of pair (block b, step t) at the trajectory state['x']."""
    sc, part, obs, nrow, yoff, tot = layout if layout is not None else workloads.block_layout(prob)
    i, j, s = part[b], obs[b], sc[b]
    pf, of = prob["part_face_ptr"], prob["obs_face_ptr"]
    A = prob["part_A"][pf[i]:pf[i + 1]]
    bb = prob["part_b"][pf[i]:pf[i + 1]]
    C = prob["obs_C"][of[j]:of[j + 1]]
    d = prob["obs_d"][of[j]:of[j + 1]]
    xs = state["x"][s, t]
    R = rotation(prob, xs)
    pos = xs[list(prob["pos_idx"])] + R @ prob["part_off"][i]
    return A, bb, C @ R, d - C @ pos


def K_rows(A, Cp, dp):
    nr, no, dim = len(A), len(dp), A.shape[1]
    K = np.zeros((nr + no + 1, dim + 1))
    K[:nr, 1:] = A
    K[nr:nr + no, 0] = dp
    K[nr:nr + no, 1:] = Cp
    K[-1, 0] = 1.0
    return K


def gather_pairs(prob, state, pairs, layout=None):
    """Stateless-batch arrays for the listed (block, t) pairs of an iterate."""
    layout = layout if layout is not None else workloads.block_layout(prob)
    sc, part, obs, nrow, yoff, tot = layout
    N, dim = prob["N"], prob["dim"]
    row_ptr = [0]
    K, kap, yh, bh, geo = [], [], [], [], []
    for (b, t) in pairs:
        A, bb, Cp, dp = pair_geometry(prob, state, b, t, layout)
        Kb = K_rows(A, Cp, dp)
        K.append(Kb)
        kap.append(np.r_[bb, np.zeros(len(dp) + 1)])
        yh.append(state["y"][yoff[b] + np.arange(nrow[b]) * N + t - 1])
        z = state["zeta"][b * N + t - 1]
        xi = state["xi"][(b * dim + np.arange(dim)) * N + t - 1]
        bh.append(np.r_[1.0 + z, xi])
        row_ptr.append(row_ptr[-1] + len(Kb))
        geo.append((A, bb, Cp, dp, z, xi))
    return (np.asarray(row_ptr, np.int32), np.concatenate(K), np.concatenate(kap), np.concatenate(yh),
            np.asarray(bh), geo)


def scaled_pair_error(K, y_test, y_ref):
    """||sqrt(D) (y_test - y_ref)|| / max(||sqrt(D) y_ref||, 1), D_l = ||K_l||^2:
    the error in the variables the proximal term makes comparable across rows."""
    w = np.sqrt((K ** 2).sum(1))
    return np.linalg.norm(w * (y_test - y_ref)) / max(np.linalg.norm(w * y_ref), 1.0)


def per_pair_y_errors(prob, y_test, y_ref, K_of_pair=None):
    """Scaled error of every pair of two canonical y vectors (weights from the
    reference iterate's geometry are not needed when K_of_pair is None: plain
    relative error per pair)."""
    sc, part, obs, nrow, yoff, tot = workloads.block_layout(prob)
    N = prob["N"]
    errs = []
    for b in range(len(sc)):
        blk_t = y_test[yoff[b]:yoff[b] + nrow[b] * N].reshape(nrow[b], N)
        blk_r = y_ref[yoff[b]:yoff[b] + nrow[b] * N].reshape(nrow[b], N)
        num = np.linalg.norm(blk_t - blk_r, axis=0)
        den = np.maximum(np.linalg.norm(blk_r, axis=0), 1.0)
        errs.append(num / den)
    return np.concatenate(errs) if errs else np.zeros(0)


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-30)


def row_weights(prob, x):
    """sqrt(D_l) = ||row_l K|| for every dual entry of the canonical y layout at
    trajectory x (vectorised over t per block)."""
    sc, part, obs, nrow, yoff, tot = workloads.block_layout(prob)
    N, dim = prob["N"], prob["dim"]
    pf, of = prob["part_face_ptr"], prob["obs_face_ptr"]
    w = np.zeros(tot)
    for b in range(len(sc)):
        i, j, s = part[b], obs[b], sc[b]
        A = prob["part_A"][pf[i]:pf[i + 1]]
        C = prob["obs_C"][of[j]:of[j + 1]]
        d = prob["obs_d"][of[j]:of[j + 1]]
        pos = np.stack([x[s, t][list(prob["pos_idx"])] + rotation(prob, x[s, t]) @ prob["part_off"][i]
                        for t in range(1, N + 1)])          # N x dim
        dp = d[None, :] - pos @ C.T                          # N x n_o
        rows = np.concatenate([np.repeat(np.linalg.norm(A, axis=1)[:, None], N, 1),
                               np.sqrt(dp.T ** 2 + (C ** 2).sum(1)[:, None]),
                               np.ones((1, N))])
        w[yoff[b]:yoff[b] + nrow[b] * N] = rows.ravel()
    return w


def scaled_y_errors(prob, x, y_test, y_ref):
    """Per-pair ||sqrt(D)(y_test - y_ref)|| / max(||sqrt(D) y_ref||, 1)."""
    sc, part, obs, nrow, yoff, tot = workloads.block_layout(prob)
    N = prob["N"]
    w = row_weights(prob, x)
    errs = []
    for b in range(len(sc)):
        sl = slice(yoff[b], yoff[b] + nrow[b] * N)
        wt = (w[sl] * y_test[sl]).reshape(nrow[b], N)
        wr = (w[sl] * y_ref[sl]).reshape(nrow[b], N)
        errs.append(np.linalg.norm(wt - wr, axis=0) / np.maximum(np.linalg.norm(wr, axis=0), 1.0))
    return np.concatenate(errs) if errs else np.zeros(0)


def multiplier_scale(prob, x, y):
    """Per-pair magnitude of the terms summed in T and R: 1 + sum_l ||K_l||_1 y_l
    (the scale FP32 rounding of T, R and of the pose acts on)."""
    sc, part, obs, nrow, yoff, tot = workloads.block_layout(prob)
    N = prob["N"]
    w = row_weights(prob, x) * np.sqrt(prob["dim"] + 1)
    out = []
    for b in range(len(sc)):
        sl = slice(yoff[b], yoff[b] + nrow[b] * N)
        out.append(1.0 + (w[sl] * np.abs(y[sl])).reshape(nrow[b], N).sum(0))
    return np.concatenate(out) if out else np.zeros(0)


def traj_error(g, o):
    """Normwise relative error over (x, u) of every scenario; the max."""
    errs = []
    for s in range(o["x"].shape[0]):
        a = np.concatenate([g["x"][s].ravel(), g["u"][s].ravel()])
        b = np.concatenate([o["x"][s].ravel(), o["u"][s].ravel()])
        errs.append(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))
    return max(errs)
