"""Independent reference for the multipole pins: every site (q, mu, Theta) is
replaced by a small cluster of point charges with the same charge, dipole and
(traceless) second moment, and the Coulomb sums are evaluated in 80-digit
arithmetic (mpmath).  Only Coulomb's law is used, none of the oracle's
multipole algebra.

Convention matched: the potential of a site is [q - mu.grad + Theta:grad grad] 1/r,
i.e. Theta = (1/2) sum_k q_k s_k s_k (traceless part) of its charge cluster.
"""
import mpmath as mp
import numpy as np

mp.mp.dps = 80
H = mp.mpf("1e-12")


def cluster(pos, m):
    """Point charges [(q, x, y, z)] representing site m at pos."""
    p = [mp.mpf(float(v)) for v in pos]
    out = []
    q = mp.mpf(float(m[0]))
    if q != 0:
        out.append((q, *p))
    mu = np.array(m[1:4], dtype=float)
    nm = float(np.linalg.norm(mu))
    if nm > 0:
        e = [mp.mpf(float(v)) / mp.mpf(nm) for v in mu]
        Q = mp.mpf(nm) / H
        out.append((Q, *[p[a] + H / 2 * e[a] for a in range(3)]))
        out.append((-Q, *[p[a] - H / 2 * e[a] for a in range(3)]))
    T = np.array([[m[4], m[5], m[6]], [m[5], m[7], m[8]], [m[6], m[8], m[9]]], dtype=float)
    if np.any(T != 0):
        lam, vec = np.linalg.eigh(T)
        for k in range(3):
            L = mp.mpf(float(lam[k]))
            if L == 0:
                continue
            e = [mp.mpf(float(v)) for v in vec[:, k]]
            Q = L / H ** 2
            out.append((Q, *[p[a] + H * e[a] for a in range(3)]))
            out.append((Q, *[p[a] - H * e[a] for a in range(3)]))
            out.append((-2 * Q, *p))
    return out


def coulomb_energy(ci, cj, coulomb):
    s = mp.mpf(0)
    for (qa, xa, ya, za) in ci:
        for (qb, xb, yb, zb) in cj:
            s += qa * qb / mp.sqrt((xa - xb) ** 2 + (ya - yb) ** 2 + (za - zb) ** 2)
    return float(s * mp.mpf(coulomb))


def field_at(point, cj):
    p = [mp.mpf(float(v)) for v in point]
    E = [mp.mpf(0)] * 3
    for (qb, xb, yb, zb) in cj:
        d = [p[0] - xb, p[1] - yb, p[2] - zb]
        r = mp.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
        for a in range(3):
            E[a] += qb * d[a] / r ** 3
    return np.array([float(v) for v in E])
