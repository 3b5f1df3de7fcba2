"""Brute-force sampled tracer for tiny grids.

An independent check of the oracle's cell-crossing geometry, splitting and
deposits: each ray is sampled at midpoints r + (k + 1/2) h, every sample is
assigned to the leaf cell holding it, consecutive samples in one cell form a
segment, the split test (section 2.1, Eq. split) is applied at the sampled exit
radius of each segment, and photons are removed by sub-stepped Beer-Lambert
attenuation over the sampled length (section 2.2, Eqs. dtau, flux). No cell
boundary is ever intersected analytically.
"""
from __future__ import annotations

import math

import numpy as np


class Hierarchy:
    def __init__(self, problem):
        self.p = problem
        self.root = problem.grids[0]
        nz, ny, nx = self.root.n_h.shape
        self.N = np.array([nx, ny, nz])
        self.cover = -np.ones((nz, ny, nx), dtype=np.int64)
        self.offs = [0]
        for g in problem.grids:
            self.offs.append(self.offs[-1] + g.n_h.size)
        for q, g in enumerate(problem.grids[1:], start=1):
            o = g.offset
            gz, gy, gx = g.n_h.shape
            self.cover[o[2]:o[2] + gz // 2, o[1]:o[1] + gy // 2, o[0]:o[0] + gx // 2] = q

    def leaf(self, pts: np.ndarray):
        """(leaf id in the concatenated cell numbering or -1, grid index)."""
        c = np.floor(pts).astype(np.int64)
        inside = np.all((c >= 0) & (c < self.N), axis=1)
        lid = -np.ones(len(pts), dtype=np.int64)
        gid = -np.ones(len(pts), dtype=np.int64)
        ci = c[inside]
        nx, ny, _ = self.N
        q = self.cover[ci[:, 2], ci[:, 1], ci[:, 0]]
        ids = np.empty(len(ci), dtype=np.int64)
        root = q < 0
        ids[root] = ci[root, 0] + nx * (ci[root, 1] + ny * ci[root, 2])
        qs = np.where(root, 0, q)
        for qq in np.unique(q[~root]):
            g = self.p.grids[qq]
            gz, gy, gx = g.n_h.shape
            sel = q == qq
            f = np.floor(2.0 * (pts[inside][sel] - np.asarray(g.offset, dtype=np.float64))).astype(np.int64)
            f = np.clip(f, 0, [gx - 1, gy - 1, gz - 1])
            ids[sel] = self.offs[qq] + f[:, 0] + gx * (f[:, 1] + gy * f[:, 2])
        lid[inside] = ids
        gid[inside] = qs
        return lid, gid


def trace(problem, pix2vec, h: float = 1e-4):
    """Returns absorbed per leaf cell, summed P at segment entry per leaf cell,
    escaped and truncated totals, and the number of split decisions within 2h
    of the threshold (ambiguous for sampling)."""
    H = Hierarchy(problem)
    grids = problem.grids
    nabs = np.concatenate([(g.n_h.astype(np.float64) * g.x_hi.astype(np.float64)).ravel() for g in grids])
    dx_root = grids[0].dx_cm
    ncell = len(nabs)
    absorbed = np.zeros(ncell)
    visits = np.zeros(ncell)
    escaped = truncated = 0.0
    ambiguous = 0
    par = problem.params
    sp = problem.spectrum
    four_pi_phi = 4.0 * math.pi * par.phi_c
    tmax_box = float(np.linalg.norm(H.N)) + 2.0
    for s_row in np.asarray(problem.sources):
        s = s_row[:3]
        for gi in range(sp.n_groups):
            sigma = sp.sigma_cm2[gi]
            n0 = 12 * 4 ** par.level_init
            P0 = sp.frac[gi] * s_row[3] / n0
            stack = [(par.level_init, p, 0.0, P0, P0) for p in reversed(range(n0))]
            while stack:
                lev, pix, r, P, Pref = stack.pop()
                n = pix2vec(lev, pix)
                if lev < par.level_max and par.phi_c > 0:
                    t_thr = math.sqrt(12.0 * 4 ** lev / four_pi_phi)   # in local cells
                    t_lim = min(tmax_box, t_thr + 2.0)
                else:
                    t_thr, t_lim = None, tmax_box
                k = max(1, int(math.ceil((t_lim - r) / h)))
                ts = r + (np.arange(k) + 0.5) * h
                lid, gid = H.leaf(s[None, :] + ts[:, None] * n[None, :])
                brk = np.flatnonzero(np.diff(lid)) + 1
                starts = np.concatenate([[0], brk])
                ends = np.concatenate([brk, [k]])
                done = False
                for j, (a, b) in enumerate(zip(starts, ends)):
                    cell = lid[a]
                    if cell < 0:
                        escaped += P
                        done = True
                        break
                    scale = 1.0 if gid[a] == 0 else 2.0
                    te = ts[b - 1] + 0.5 * h
                    r_in = r if j == 0 else ts[a] - 0.5 * h
                    if t_thr is not None:
                        if abs(te * scale - t_thr) < 2.0 * h * scale:
                            ambiguous += 1
                        if 12.0 * 4 ** lev < four_pi_phi * (te * scale) ** 2:
                            for kk in (3, 2, 1, 0):
                                stack.append((lev + 1, 4 * pix + kk, r_in, 0.25 * P, 0.25 * Pref))
                            done = True
                            break
                    if b == k:
                        raise RuntimeError("sampling window ended inside the grid")
                    L = (b - a) * h * dx_root
                    tau = sigma * nabs[cell] * L
                    dP = P * (-math.expm1(-tau))
                    absorbed[cell] += dP
                    visits[cell] += P
                    P -= dP
                    if P < par.p_min_frac * Pref:
                        truncated += P
                        done = True
                        break
                if not done:
                    raise RuntimeError("ray neither ended nor split inside its sampling window")
    return {"absorbed": absorbed, "visits": visits, "escaped": escaped, "truncated": truncated,
            "ambiguous": ambiguous, "kappa_root": sp.sigma_cm2.max() * nabs.max() * dx_root}
