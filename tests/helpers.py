"""Test helpers: block-level pairing, comparisons and tiny problems (no method arithmetic
beyond the bilinear pairing used by the adjoint identity)."""
import numpy as np

from paper_2202_08612_amd import inputs as I


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0))


def maxrel(a, b):
    mb = np.max(np.abs(b)) if np.size(b) else 0.0
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / (mb if mb > 0 else 1.0)) if np.size(b) else 0.0


def packed_masks(d):
    a = np.arange(d.n_v)[:, None, None, None]
    D = np.arange(d.N_V)[None, :, None, None]
    i = np.arange(d.n_o)[None, None, :, None]
    j = np.arange(d.n_o)[None, None, None, :]
    m1 = (D >= d.n_v) | (a * d.N_O + i >= D * d.N_O + j)
    L = np.arange(d.N_O)[None, None, None, :]
    m2 = np.broadcast_to(L >= d.n_o, (d.n_v, d.n_v, d.n_o, d.N_O))
    return np.broadcast_to(m1, (d.n_v, d.N_V, d.n_o, d.n_o)), m2


def swapped_virtuals(d, X):
    """X^{BA}_{IJ} on both blocks of a pair-symmetric doubles array given as blocks."""
    A = X["x2_vVoo"]
    Bv = X["x2_vvoO"]
    sa = np.empty_like(A)
    # D inactive: X^{Da}_{ij} = X^{aD}_{ji}; D active: X^{Da}_{ij} from the block directly
    sa[:, :, :, :] = np.einsum("adji->adij", A)
    sa[:, :d.n_v] = np.einsum("daij->adij", A[:, :d.n_v])
    sb = np.einsum("bail->abil", Bv)
    return sa, sb


def pair_form_blocks(d, X, Y):
    """G(X,Y) = sum X1 Y1 + sum_{(AI)>=(BJ)} X~2 Y2 on the union of the two blocks."""
    m1, m2 = packed_masks(d)
    sa, sb = swapped_virtuals(d, X)
    Xa = 2.0 * X["x2_vVoo"] - sa
    Xb = 2.0 * X["x2_vvoO"] - sb
    return float(np.sum(X["x1"] * Y["x1"]) + np.sum(np.where(m1, Xa * Y["x2_vVoo"], 0.0))
                 + np.sum(np.where(m2, Xb * Y["x2_vvoO"], 0.0)))


def vec_lin(a, x, b, y):
    return {k: a * x[k] + b * y[k] for k in x}


def rbar_blocks(d, R):
    """(1 + delta_{ai,bj}) R on both blocks."""
    A = R["x2_vVoo"].copy()
    for a in range(d.n_v):
        for i in range(d.n_o):
            A[a, a, i, i] *= 2.0
    B = R["x2_vvoO"].copy()
    for a in range(d.n_v):
        for i in range(d.n_o):
            B[a, a, i, i] *= 2.0
    return A, B


def compare_out(o, ref):
    return {k: rel(o[k], ref[k]) for k in ("x1", "x2_vVoo", "x2_vvoO")}


# ------------------------------------------------- pairing maps (for gradient tests)
def _amp_index(d):
    """For every stored doubles position (block x2_vVoo then x2_vvoO, row-major) the index of its
    amplitude {(A,I),(B,J)} and of the virtual-swapped amplitude X^{BA}_{IJ} in one numbering."""
    A1, B1, I1, J1 = np.meshgrid(np.arange(d.n_v), np.arange(d.N_V), np.arange(d.n_o), np.arange(d.n_o),
                                 indexing="ij")
    A2, B2, I2, J2 = np.meshgrid(np.arange(d.n_v), np.arange(d.n_v), np.arange(d.n_o), np.arange(d.N_O),
                                 indexing="ij")
    A = np.concatenate([A1.ravel(), A2.ravel()])
    B = np.concatenate([B1.ravel(), B2.ravel()])
    Ii = np.concatenate([I1.ravel(), I2.ravel()])
    J = np.concatenate([J1.ravel(), J2.ravel()])
    npair = d.N_V * d.N_O

    def key(a, i, b, j):
        p, q = a * d.N_O + i, b * d.N_O + j
        return np.minimum(p, q) * npair + np.maximum(p, q)

    n = A.size
    _, inv = np.unique(np.concatenate([key(A, Ii, B, J), key(B, Ii, A, J)]), return_inverse=True)
    return inv[:n], inv[n:], int(inv.max()) + 1, A1.size


def _split(d, flat, nA):
    return flat[:nA].reshape(d.n_v, d.N_V, d.n_o, d.n_o), flat[nA:].reshape(d.n_v, d.n_v, d.n_o, d.N_O)


def map_symmetrize(d, X):
    ids, _, nu, nA = _amp_index(d)
    flat = np.concatenate([X["x2_vVoo"].ravel(), X["x2_vvoO"].ravel()])
    mean = np.bincount(ids, weights=flat, minlength=nu) / np.maximum(np.bincount(ids, minlength=nu), 1)
    a, b = _split(d, mean[ids], nA)
    return {"x1": X["x1"].copy(), "x2_vVoo": a, "x2_vvoO": b}


def map_grad_to_left(d, g):
    """L with G(L, y) = <g, y> for consistent y: L = (2 s + s^{BA}_{IJ}) / 3, s = sum over positions."""
    ids, sw, nu, nA = _amp_index(d)
    flat = np.concatenate([g["x2_vVoo"].ravel(), g["x2_vvoO"].ravel()])
    s = np.bincount(ids, weights=flat, minlength=nu)
    a, b = _split(d, (2.0 * s[ids] + s[sw]) / 3.0, nA)
    return {"x1": g["x1"].copy(), "x2_vVoo": a, "x2_vvoO": b}


def map_left_to_grad(d, S):
    """h with <h, y> = G(S, y) for consistent y, spread evenly over the stored positions."""
    ids, sw, nu, nA = _amp_index(d)
    flat = np.concatenate([S["x2_vVoo"].ravel(), S["x2_vvoO"].ravel()])
    cnt = np.bincount(ids, minlength=nu)
    val = np.bincount(ids, weights=flat, minlength=nu) / np.maximum(cnt, 1)
    a, b = _split(d, (2.0 * flat - val[sw]) / cnt[ids], nA)
    return {"x1": S["x1"].copy(), "x2_vVoo": a, "x2_vvoO": b}


def euclid(x, y):
    return float(sum(np.sum(np.asarray(x[k]) * np.asarray(y[k])) for k in ("x1", "x2_vVoo", "x2_vvoO")))
