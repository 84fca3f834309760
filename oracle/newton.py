"""Hessian, Kantorovich functional and damped Newton solve (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Derivatives of the semi-discrete dual K(psi) of Eq. SDK (the paper states that
K is concave and C^2 and maximised by a Newton method using its first and
second derivatives; the derivatives themselves are not printed and are
derived here from Eq. SDK and Eq. laguerrecell):

  dK/dpsi_i = m_i - |V_i|         (the envelope min_i pi_i has slope -1 on V_i)
  J := dV/dpsi = -Hess K:          J_ij = -sum_images A_ij / |d_ij|  (j != i),
                                   J_ii = -sum_{j != i} J_ij
  (raising psi_j by t moves the common face towards x_i by t/|d_ij|.)

Newton for V(psi) = m solves  J p = m - V.  Step control follows Kitagawa,
Merigot and Thibert (the reference the paper gives for convergence):
eps0 = 1/2 min(min_i m_i, min_i |V_i(psi^0)|); the step 2^-l p is accepted
for the smallest l with min_i |V_i| >= eps0 and
||m - V||_2 <= (1 - 2^-(l+1)) ||m - V(psi^k)||_2.
Masses default to uniform, m_i = L^3 / N (initial density 1, sum m_i = L^3);
solve() also takes one target mass per site (Eq. SDK with weighted sites).
"""
from __future__ import annotations

import numpy as np

from .cells import cells


def _coo_entries(res: dict, n: int):
    """(row, col, value) triples of the off-diagonal entries -A/|d| (one per
    face; images of the same j are separate triples, summed later)."""
    rows, cols, vals = [], [], []
    fp = res["face_ptr"]
    for k in range(len(res["idx"])):
        i = int(res["idx"][k])
        for f in range(fp[k], fp[k + 1]):
            j = int(res["face_j"][f])
            if j == i:
                continue  # faces of the own-image box do not move with psi
            rows.append(i)
            cols.append(j)
            vals.append(-res["face_area"][f] / res["face_dist"][f])
    return np.array(rows, dtype=np.int64), np.array(cols, dtype=np.int64), np.array(vals)


def hessian_coo(res: dict, n: int):
    """Sparse J = dV/dpsi as a scipy CSR matrix (sum of images, diagonal =
    minus the off-diagonal row sum)."""
    import scipy.sparse as sp
    r, c, v = _coo_entries(res, n)
    off = sp.coo_matrix((v, (r, c)), shape=(n, n)).tocsr()
    off.sum_duplicates()
    diag = -np.asarray(off.sum(axis=1)).ravel()
    return (off + sp.diags(diag)).tocsr()


def hessian_dense(res: dict, n: int) -> np.ndarray:
    r, c, v = _coo_entries(res, n)
    J = np.zeros((n, n))
    np.add.at(J, (r, c), v)
    J[np.arange(n), np.arange(n)] = -J.sum(axis=1)
    return J


def kantorovich(res: dict, psi, m) -> float:
    """K(psi) = sum_i int_{V_i} (1/2 |x_i - q|^2 - psi_i) dq + sum_i m_i psi_i
    (Eq. SDK), from the second moments S_i and volumes."""
    psi = np.asarray(psi, dtype=np.float64)
    return float(np.sum(0.5 * res["S"] - psi * res["V"]) + np.sum(np.asarray(m) * psi))


def centroids_from_moments(x, res: dict, L: float):
    """Cell centroids wrapped into [0, L)^3 and displacements x_i - c_i
    (= minus the seed-local centroid, so no wrap ambiguity)."""
    V = res["V"]
    u = np.where(V[:, None] > 0, res["M"] / np.where(V > 0, V, 1.0)[:, None], 0.0)
    c = np.mod(np.asarray(x) + u, L)
    c[c >= L] = 0.0
    return c, -u


def newton_step_dense(J: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Solve J p = g on the complement of the constants: (J + c 1 1^T) p = g
    with c = mean(diag J) / N, which gives the mean-zero solution when
    sum(g) = 0 (J is a connected graph Laplacian)."""
    n = J.shape[0]
    g = g - g.mean()
    c = float(np.mean(np.diag(J))) / n
    return np.linalg.solve(J + c * np.ones((n, n)), g)


def newton_step_cg(J, g: np.ndarray, rtol: float = 1e-12, maxiter: int | None = None) -> np.ndarray:
    """Plain conjugate gradients for J p = g restricted to mean-zero vectors."""
    n = g.shape[0]
    b = g - g.mean()
    p = np.zeros(n)
    r = b.copy()
    d = r.copy()
    rr = float(r @ r)
    stop = (rtol ** 2) * float(b @ b)
    maxiter = maxiter or 10 * n
    for _ in range(maxiter):
        if rr <= stop:
            break
        q = J @ d
        a = rr / float(d @ q)
        p += a * d
        r -= a * q
        r -= r.mean()
        rr_new = float(r @ r)
        d = r + (rr_new / rr) * d
        rr = rr_new
    return p - p.mean()


def solve(x, L: float, tol: float = 1e-6, max_newton: int = 50, threads: int = 0,
          dense_max: int = 4096, psi0=None, log=None, masses=None) -> dict:
    """Damped Newton maximisation of K(psi) until max_i |V_i - m_i| / m_i <= tol.

    masses: target volume per site (positive, summing to L^3); uniform
    L^3 / N when omitted.  Returns psi (mean zero), centroids, displacements,
    the final cell result and iteration statistics."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.shape[0]
    if masses is None:
        m = np.full(n, L ** 3 / n)
    else:
        m = np.array(masses, dtype=np.float64).reshape(n)
        if not (np.all(m > 0) and abs(m.sum() - L ** 3) <= 1e-9 * L ** 3):
            raise ValueError("masses must be positive and sum to L^3")
    psi = np.zeros(n) if psi0 is None else np.array(psi0, dtype=np.float64)
    res = cells(x, psi, L, threads=threads)
    if np.any(res["flags"] & 2):
        raise ValueError("coincident sites")
    eps0 = 0.5 * min(float(m.min()), float(res["V"].min()))
    stats = {"newton_iters": 0, "ls_trials": 0, "errs": []}
    for it in range(max_newton + 1):
        g = m - res["V"]
        err = float(np.max(np.abs(g) / m))
        stats["errs"].append(err)
        if log is not None:
            log(it, err)
        if err <= tol:
            break
        if it == max_newton:
            raise RuntimeError(f"Newton did not converge: err={err}")
        if n <= dense_max:
            p = newton_step_dense(hessian_dense(res, n), g)
        else:
            p = newton_step_cg(hessian_coo(res, n), g)
        gn = float(np.linalg.norm(g))
        alpha = 1.0
        for _ls in range(31):
            trial = psi + alpha * p
            rt = cells(x, trial, L, threads=threads)
            stats["ls_trials"] += 1
            ok = (not np.any(rt["flags"] & 1)) and float(rt["V"].min()) >= eps0
            if ok and float(np.linalg.norm(m - rt["V"])) <= (1.0 - 0.5 * alpha) * gn:
                break
            alpha *= 0.5
        else:
            raise RuntimeError("line search failed")
        psi, res = trial, rt
        stats["newton_iters"] += 1
    c, disp = centroids_from_moments(x, res, L)
    return {"psi": psi - psi.mean(), "centroids": c, "disp": disp, "res": res,
            "err": stats["errs"][-1], **stats}
