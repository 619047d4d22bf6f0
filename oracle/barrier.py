"""Energy barrier by the simplified string method, and BER_adj -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the bench's CPU baseline may import this module.

The paper obtains the energy barrier E_B of the adjacent bit, in the head's fringing field at the
down-track position 2 nm from the trailing edge, with a minimum-energy-path method (nudged
elastic band) and turns it into BER_adj = t_write f0 exp(-E_B / kB T) (Sec. II.C, Eq. (3),
f0 = 130 GHz, t_write = 1 ns, T = 300 K).  The oracle computes the minimum energy path with the
simplified string method (E, Ren and Vanden-Eijnden, J. Chem. Phys. 126, 164103 (2007)):

1. a chain of P images of the island's magnetisation, from the stored state to the reversed one;
2. every iteration first relaxes each image for a pseudo-time dtau along the damping term of the
   LLG equation alone (the oracle's own DP5 integrator with the precession term dropped), which
   moves it down the total energy;
3. then puts the images back at equal spacing along the chain: with d_k the Euclidean distance of
   images k and k+1 over all 3n node components and s_k the summed distance up to image k, image
   j moves to s = j s_{P-1} / (P-1), linearly interpolated between the two images that bracket
   it, every node vector normalised again (the end images keep their place);
4. after the last iteration, the energies E_k of the relaxed images at their arc lengths s_k give
   E_B = max_k E_k - E_0; an interior maximum is refined by the vertex of the parabola through it
   and its two neighbours in (s, E).
"""
from __future__ import annotations

import math

import numpy as np

KB = 1.380649e-23
F0 = 130e9
T_WRITE = 1e-9


def rotation_chain(n: int, P: int, via=(1.0, 0.0, 0.0)) -> np.ndarray:
    """P uniform states turning from +z to -z through the unit direction `via` (perpendicular to
    z): image k at polar angle pi k / (P - 1).  Returns [P][3][n]."""
    v = np.asarray(via, dtype=np.float64)
    out = np.empty((P, 3, n))
    for k in range(P):
        th = math.pi * k / (P - 1)
        d = math.cos(th) * np.array([0.0, 0.0, 1.0]) + math.sin(th) * v
        out[k] = d[:, None]
    return out


def redistribute(imgs: np.ndarray):
    """Step 3: images [P][3][n] back to equal arc length.  Returns (new images, arc lengths of the
    given images)."""
    P = imgs.shape[0]
    d = np.array([np.linalg.norm((imgs[k + 1] - imgs[k]).ravel()) for k in range(P - 1)])
    s = np.concatenate([[0.0], np.cumsum(d)])
    out = np.empty_like(imgs)
    out[0] = imgs[0]
    out[P - 1] = imgs[P - 1]
    for j in range(1, P - 1):
        target = s[-1] * j / (P - 1)
        k = int(np.searchsorted(s, target, side="right")) - 1
        k = min(max(k, 0), P - 2)
        w = (target - s[k]) / d[k] if d[k] > 0 else 0.0
        w = min(1.0, max(0.0, w))
        v = (1.0 - w) * imgs[k] + w * imgs[k + 1]
        out[j] = v / np.linalg.norm(v, axis=0)
    return out, s


def barrier_of_profile(s, E) -> float:
    """Step 4: E_B from the energies E_k at arc lengths s_k."""
    s = np.asarray(s, dtype=np.float64)
    E = np.asarray(E, dtype=np.float64)
    k = int(np.argmax(E))
    top = E[k]
    if 0 < k < len(E) - 1:
        # vertex of the parabola through (s_{k-1}, E_{k-1}), (s_k, E_k), (s_{k+1}, E_{k+1})
        x0, x1, x2 = s[k - 1], s[k], s[k + 1]
        y0, y1, y2 = E[k - 1], E[k], E[k + 1]
        den = (x0 - x1) * (x0 - x2) * (x1 - x2)
        a = (x2 * (y1 - y0) + x1 * (y0 - y2) + x0 * (y2 - y1)) / den
        b = (x2 * x2 * (y0 - y1) + x1 * x1 * (y2 - y0) + x0 * x0 * (y1 - y2)) / den
        c = (x1 * x2 * (x1 - x2) * y0 + x2 * x0 * (x2 - x0) * y1 + x0 * x1 * (x0 - x1) * y2) / den
        if a < 0:
            xv = -b / (2 * a)
            if x0 <= xv <= x2:
                top = max(top, c - b * b / (4 * a))
    return float(top - E[0])


def string_barrier(om, S, mat, fld, chain, offset=(0.0, 0.0, 0.0), dtau: float = 2e-12, iters: int = 60,
                   rtol: float = 1e-6):
    """Runs the string method from `chain` [P][3][n].  Returns dict(E_B, energies, arclen,
    images) of the last relaxed chain."""
    imgs = np.array(chain, dtype=np.float64)
    P = imgs.shape[0]
    offs = np.broadcast_to(np.asarray(offset, dtype=np.float64), (P, 3))
    E = s = relaxed = None
    for _ in range(iters):
        relaxed, res, _ = om.run(S, [mat] * P, [fld] * P, dict(t_end=dtau, rtol=rtol, relax=True), m0=imgs,
                                 offsets=offs)
        if any(r["status"] != 0 for r in res):
            raise RuntimeError("relaxation failed")
        E = np.array([r["energy"] for r in res])
        imgs, s = redistribute(relaxed)
    return dict(E_B=barrier_of_profile(s, E), energies=E, arclen=s, images=relaxed, next_chain=imgs)


def ber_adj(E_B: float, T: float = 300.0, f0: float = F0, t_write: float = T_WRITE) -> float:
    """Eq. (3): BER_adj = t_write / tau with tau = exp(E_B / kB T) / f0."""
    return t_write * f0 * math.exp(-E_B / (KB * T))
