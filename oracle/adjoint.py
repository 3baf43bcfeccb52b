"""Reference derivatives of the coupled lattice-Boltzmann / Brownian-particle map.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): the test-suite uses it
to check the GPU adjoint; the GPU product path never imports it.

What is differentiated.  S_N maps the state at step n0 -- post-streaming
populations f (section 2.2, Eq. s2-trans), particle positions r and velocities
V -- and the parameters theta = (gamma, tau, M, kT) to the state N steps later,
one step being the oracle's order: moments (Eqs. s2-density, s2-fv), friction
F_H from the eight nodes around each particle (Eq. s2-slet-v, or Eq. s2-dis1 /
Eq. s2-dis0), Brownian force F_R = sqrt(2 gamma kT) xi (Eqs. s2-rf1, s2-rf2),
spreading of -F_H with trilinear weights (first Eq. s2-force), BGK collision
with the forcing term (Eqs. s2-collision, s2-eq, second Eq. s2-force),
streaming, and the Langevin update V' = V + (F_H + F_R)/M, r' = r + V' (Eqs.
s2-langevin, s2-langevin2).  The particle radius is either given or follows
from Stokes' law R = gamma / (6 pi eta), eta = (tau - 1/2)/3 (Eq. s2-ident3),
in which case it moves with gamma and tau.  The normals xi are inputs (drawn
by the oracle's Philox generator), so the map is deterministic and the
derivative is the pathwise one.  The corner cell floor(s) and the branch
tests (zero mean relative velocity, zero fit denominator, a node on the
particle) are piecewise constant and differentiate to zero.

How.  ``run`` is a plain numpy transcription of that step, written so that the
same code evaluates in float64 and in complex128.  Then

* ``jvp`` -- directional derivative by the complex step (Squire & Trapp,
  SIAM Review 1998): d/dh J(x + i h v) at h -> 0 equals Im J(x + i h v) / h
  with no subtractive cancellation, i.e. exact up to rounding;
* ``vjp`` -- the gradient of <c, S_N(x)> by a reverse sweep over the stored
  trajectory in which every local Jacobian (the collision at each node, the
  particle update as a function of its eight corner nodes) is itself obtained
  column by column with the complex step.  No derivative formula is written
  out anywhere in this file.

Trilinear weights.  Within the corner cell c = floor(s) the weight factor
1 - |d| of a node offset d = c + b - s is 1 + d for b = 0 and 1 - d for
b = 1, the analytic form used here (identical to the oracle's for real d).
"""
from __future__ import annotations

import numpy as np

from . import FRICTION, gauss3, lattice

H = 1e-30  # complex-step size

_TABLES = {}


def _tables(q: int):
    """(e [q, 3] float, w [q]) of the velocity set with q = 19 or 15."""
    if q not in _TABLES:
        e, w = lattice(q)
        _TABLES[q] = (e.astype(np.float64), w)
    return _TABLES[q]
_BITS = np.array([[p & 1, (p >> 1) & 1, (p >> 2) & 1] for p in range(8)], dtype=np.int64)


def noise(n: int, nsteps: int, seed: int, step0: int = 0, replica: int = 0) -> np.ndarray:
    """The normals xi[k, i, :] of step step0 + k, particle i (Philox stream 0)."""
    xi = np.zeros((nsteps, n, 3))
    for k in range(nsteps):
        for i in range(n):
            xi[k, i] = gauss3(seed, step0 + k, i, replica, 0)
    return xi


def radius_of(theta, radius: float):
    """Particle radius: the given one, or Stokes' law from gamma and tau."""
    if radius > 0.0:
        return radius
    gamma, tau = theta[0], theta[1]
    nu = (tau - 0.5) / 3.0
    return gamma / (6.0 * np.pi * nu)


def collide(f, F, tau):
    """Post-collision populations of every node, f + (f^eq - f)/tau + 3 w e.F
    (Eqs. s2-collision, s2-eq, second Eq. s2-force): f [q, *nodes],
    F [3, *nodes]."""
    E, W = _tables(f.shape[0])
    rho = f.sum(axis=0)
    u = np.tensordot(E.T, f, axes=(1, 0))            # (3, *nodes)
    uu = (u * u).sum(axis=0)
    eu = np.tensordot(E, u, axes=(1, 0))             # (q, *nodes)
    wb = W.reshape((len(W),) + (1,) * (f.ndim - 1))
    feq = wb * (rho + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu)
    eF = np.tensordot(E, F, axes=(1, 0))
    return f + (feq - f) / tau + 3.0 * wb * eF


def stream(fs):
    """f_a(x + e_a) <- fs_a(x), periodic: fs [q, nz, ny, nx]."""
    E, _ = _tables(fs.shape[0])
    out = np.empty_like(fs)
    for a in range(fs.shape[0]):
        ex, ey, ez = (int(v) for v in E[a])
        out[a] = np.roll(fs[a], shift=(ez, ey, ex), axis=(0, 1, 2))
    return out


def corners(r, shape):
    """Corner cell of each particle from the real part of its position.
    Returns c [n, 3] (float, unwrapped cell corner in the wrapped frame) and
    node [n, 8] linear node indices (z, y, x order)."""
    nz, ny, nx = shape
    Lv = np.array([nx, ny, nz], dtype=np.float64)
    rr = np.real(r)
    s = rr - Lv * np.floor(rr / Lv)
    c = np.floor(s)
    ci = c.astype(np.int64)
    node = np.zeros((r.shape[0], 8), dtype=np.int64)
    for p in range(8):
        q = (ci + _BITS[p]) % np.array([nx, ny, nz])
        node[:, p] = (q[:, 2] * ny + q[:, 1]) * nx + q[:, 0]
    return c, node


def fit_corners(r, shape):
    """Corners of the (2 dx)^3 fitting cube: per axis c0 and c0 + 2 with
    c0 = floor(s + 1/2) - 1.  Returns c0 [n, 3] and node [n, 8]."""
    nz, ny, nx = shape
    Lv = np.array([nx, ny, nz], dtype=np.float64)
    rr = np.real(r)
    s = rr - Lv * np.floor(rr / Lv)
    c0 = np.floor(s + 0.5) - 1.0
    ci = c0.astype(np.int64)
    node = np.zeros((r.shape[0], 8), dtype=np.int64)
    for p in range(8):
        q = (ci + 2 * _BITS[p]) % np.array([nx, ny, nz])
        node[:, p] = (q[:, 2] * ny + q[:, 1]) * nx + q[:, 0]
    return c0, node


def pair_forces(r, shape, a_f: float, r_c: float):
    """Soft pair repulsion a_f (1 - |d|/r_c) d/|d| for |d| < r_c (Eq. s2-softpot
    read as the DPD conservative force), nearest periodic image; complex-safe
    (the image and the cutoff test use the real part)."""
    nz, ny, nx = shape
    Lv = np.array([nx, ny, nz], dtype=np.float64)
    n = r.shape[0]
    F = np.zeros(r.shape, dtype=np.result_type(r, np.float64))
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            d = r[i] - r[j]
            d = d - Lv * np.round(np.real(d) / Lv)
            dist = np.sqrt((d * d).sum())
            if np.real(dist) > 0.0 and np.real(dist) < r_c:
                F[i] = F[i] + a_f * (1.0 - dist / r_c) / dist * d
    return F


def particle_update(f8, V, r, theta, xi, c, shape, friction: int, radius: float, fc=None,
                    cfit=None):
    """One particle's step as a function of the populations at its eight
    fitting nodes.  Batch axes lead: f8 [B, 8, q], V, r [B, 3], theta [B, 4],
    xi [3]; c [3] is the corner cell (fixed, the spreading nodes); cfit [3] the
    (2 dx)^3 cube's first corner for the wide Stokeslet fit (f8 then holds
    those corners); fc [3] a given force F_C on the particle (None: zero).
    Returns (V', r', spread [B, 8, 3]) where spread is the force the eight
    corner-cell nodes receive."""
    nz, ny, nx = shape
    Lv = np.array([nx, ny, nz], dtype=np.float64)
    gamma, tau, M, kT = (theta[:, k] for k in range(4))
    s = r - Lv * np.floor(np.real(r) / Lv)            # wrapped position
    d = (c + _BITS)[None, :, :] - s[:, None, :]       # [B, 8, 3] node minus particle
    t = np.where(_BITS[None] == 0, 1.0 + d, 1.0 - d)  # 1 - |d| inside the cell
    Wt = t[..., 0] * t[..., 1] * t[..., 2]            # [B, 8]
    u8 = np.einsum("bpa,ak->bpk", f8, _tables(f8.shape[-1])[0])  # velocity at each node
    if friction == FRICTION["stokeslet2dx"]:
        d = (cfit + 2 * _BITS)[None, :, :] - s[:, None, :]
    if friction == FRICTION["bd"]:
        FH = -gamma[:, None] * V
    elif friction == FRICTION["pointwise"]:
        ur = np.einsum("bp,bpk->bk", Wt, u8)
        FH = -gamma[:, None] * (V - ur)
    else:
        R = radius_of((gamma, tau), radius)
        R = np.broadcast_to(R, gamma.shape)
        w = u8 - V[:, None, :]
        m = w.mean(axis=1)
        mn = np.sqrt((m * m).sum(axis=1))
        has_dir = np.real(mn) != 0.0
        mn_safe = np.where(has_dir, mn, 1.0)
        eN = m / mn_safe[:, None]
        rp = np.sqrt((d * d).sum(axis=2))              # [B, 8]
        use = np.real(rp) > 1e-12
        rp_safe = np.where(use, rp, 1.0)
        de = (d * eN[:, None, :]).sum(axis=2)
        ca = 1.0 - 3.0 * R[:, None] / (4.0 * rp_safe)
        cb = 3.0 * R[:, None] * de / (4.0 * rp_safe ** 3)
        g = ca[..., None] * eN[:, None, :] - cb[..., None] * d
        g = np.where(use[..., None], g, 0.0)
        num = (w * g).sum(axis=(1, 2))
        den = (g * g).sum(axis=(1, 2))
        ok = has_dir & (np.real(den) != 0.0)
        Uinf = num / np.where(ok, den, 1.0)
        FH = np.where(ok[:, None], gamma[:, None] * Uinf[:, None] * eN, 0.0)
    if np.all(np.real(kT) > 0.0):
        FR = np.sqrt(2.0 * gamma * kT)[:, None] * xi[None, :]
    else:
        FR = np.zeros_like(FH)
    if friction == FRICTION["bd"]:
        spread = np.zeros(Wt.shape + (3,), dtype=np.result_type(FH, Wt))
    else:
        spread = -FH[:, None, :] * Wt[..., None]
    if fc is None:
        Fsum = FH + FR
    else:
        Fsum = (fc if np.ndim(fc) == 2 else fc[None, :]) + FH + FR
    Vn = V + Fsum / M[:, None]
    rn = r + Vn
    return Vn, rn, spread


def step(f, r, V, theta, xi_k, friction: int, radius: float, fc=None, body=None, pair=None):
    """One coupled step; returns (f', r', V', F) with F the node-force field.
    fc: given force on each particle [n, 3] or None; body: uniform body force
    [3] on every node or None; pair: (a_f, r_c) of the pair repulsion or None."""
    shape = f.shape[1:]
    if pair is not None and r.shape[0]:
        fp = pair_forces(r, shape, *pair)
        fc = fp if fc is None else fc + fp
    ncell = int(np.prod(shape))
    dtype = np.result_type(f, r, V, theta)
    F = np.zeros((3, ncell), dtype=dtype)
    if body is not None:
        F += np.asarray(body, dtype=np.float64).reshape(3, 1)
    n = r.shape[0]
    Vn = np.empty_like(V, dtype=dtype)
    rn = np.empty_like(r, dtype=dtype)
    if n:
        c, node = corners(r, shape)
        cfit, nfit = fit_corners(r, shape) if friction == FRICTION["stokeslet2dx"] else (c, node)
        fl = f.reshape(f.shape[0], ncell)
        for i in range(n):
            f8 = fl[:, nfit[i]].T[None]                   # [1, 8, q]
            v1, r1, sp = particle_update(f8, V[i][None], r[i][None], theta[None], xi_k[i], c[i],
                                         shape, friction, radius, None if fc is None else fc[i],
                                         cfit[i])
            Vn[i], rn[i] = v1[0], r1[0]
            for p in range(8):
                F[:, node[i, p]] += sp[0, p]
    Fg = F.reshape((3,) + shape)
    fs = collide(f, Fg, theta[1])
    return stream(fs), rn, Vn, Fg


def run(f0, r0, V0, theta, xi, friction="stokeslet", radius=0.0, keep=False, fc=None, body=None,
        pair=None):
    """N = len(xi) steps from (f0, r0, V0) with parameters theta (gamma, tau,
    M, kT).  Returns (f, r, V) at the end, plus the per-step states (f^n, r^n,
    V^n, F^n) when keep."""
    friction = FRICTION[friction] if isinstance(friction, str) else int(friction)
    f, r, V = f0, r0, V0
    theta = np.asarray(theta)
    traj = []
    for k in range(len(xi)):
        fn, rn, Vn, F = step(f, r, V, theta, xi[k], friction, radius, fc, body, pair)
        if keep:
            traj.append((f, r, V, F))
        f, r, V = fn, rn, Vn
    return (f, r, V, traj) if keep else (f, r, V)


def jvp(f0, r0, V0, theta, xi, df, dr, dV, dtheta, friction="stokeslet", radius=0.0, fc=None,
        body=None, pair=None):
    """Directional derivative of S_N along (df, dr, dV, dtheta), complex step."""
    f, r, V = run(f0 + 1j * H * df, r0 + 1j * H * dr, V0 + 1j * H * dV,
                  np.asarray(theta) + 1j * H * np.asarray(dtheta), xi, friction, radius, fc=fc,
                  body=body, pair=pair)
    return np.imag(f) / H, np.imag(r) / H, np.imag(V) / H


def vjp(f0, r0, V0, theta, xi, cf, cr, cV, friction="stokeslet", radius=0.0, fc=None, body=None,
        pair=None):
    """Gradient of J = <cf, f^N> + <cr, r^N> + <cV, V^N> with respect to f0, r0,
    V0 and theta, by a reverse sweep with complex-step local Jacobians."""
    fr_mode = FRICTION[friction] if isinstance(friction, str) else int(friction)
    theta = np.asarray(theta, dtype=np.float64)
    _, _, _, traj = run(f0, r0, V0, theta, xi, fr_mode, radius, keep=True, fc=fc, body=body,
                        pair=pair)
    shape = f0.shape[1:]
    ncell = int(np.prod(shape))
    gf = np.array(cf, dtype=np.float64)
    gr = np.array(cr, dtype=np.float64)
    gV = np.array(cV, dtype=np.float64)
    gth = np.zeros(4)
    q = f0.shape[0]
    E, _ = _tables(q)
    eyeq = np.eye(q)
    for k in range(len(xi) - 1, -1, -1):
        f, r, V, F = traj[k]
        # streaming: f^{n+1}_a(x + e_a) = fs_a(x)  =>  gfs_a(x) = gf_a(x + e_a)
        gfs = np.empty_like(gf)
        for a in range(q):
            ex, ey, ez = (int(v) for v in E[a])
            gfs[a] = np.roll(gf[a], shift=(-ez, -ey, -ex), axis=(0, 1, 2))
        # collision, node by node: columns of d fs / d f by the complex step
        gfn = np.zeros_like(gf)
        for b in range(q):
            pert = f + 1j * H * eyeq[b].reshape(q, 1, 1, 1)
            col = np.imag(collide(pert, F.astype(complex), theta[1])) / H   # d fs_a / d f_b
            gfn[b] = (col * gfs).sum(axis=0)
        gF = np.zeros((3,) + shape)
        for kk in range(3):
            dF = np.zeros((3,) + shape, dtype=complex)
            dF[kk] = 1j * H
            col = np.imag(collide(f.astype(complex), F + dF, theta[1])) / H
            gF[kk] = (col * gfs).sum(axis=0)
        col = np.imag(collide(f.astype(complex), F.astype(complex), theta[1] + 1j * H)) / H
        gth[1] += (col * gfs).sum()
        # particles: columns of d(V', r', spread)/d(f8, V, r, theta)
        n = r.shape[0]
        if n:
            c, node = corners(r, shape)
            wide = fr_mode == FRICTION["stokeslet2dx"]
            cfit, nfit = fit_corners(r, shape) if wide else (c, node)
            fl = f.reshape(q, ncell)
            gFl = gF.reshape(3, ncell)
            gfl = gfn.reshape(q, ncell)
            new_gr = np.zeros_like(gr)
            new_gV = np.zeros_like(gV)
            fstep = np.zeros((n, 3)) if fc is None else np.array(fc, dtype=np.float64)
            if pair is not None:
                fstep = fstep + pair_forces(r, shape, *pair)
            gfc = np.zeros((n, 3))
            for i in range(n):
                f8 = fl[:, nfit[i]].T                      # [8, q]
                nq = 8 * q
                nin = nq + 3 + 3 + 4 + 3
                base = np.concatenate([f8.ravel(), V[i], r[i], theta, fstep[i]]).astype(complex)
                X = np.tile(base, (nin, 1)) + 1j * H * np.eye(nin)
                v1, r1, sp = particle_update(X[:, :nq].reshape(nin, 8, q), X[:, nq:nq + 3],
                                             X[:, nq + 3:nq + 6], X[:, nq + 6:nq + 10], xi[k][i],
                                             c[i], shape, fr_mode, radius, X[:, nq + 10:nq + 13],
                                             cfit[i])
                jv, jr, jsp = np.imag(v1) / H, np.imag(r1) / H, np.imag(sp) / H
                ybar_sp = gFl[:, node[i]].T                # [8, 3] gradient of each node force
                xbar = jv @ gV[i] + jr @ gr[i] + np.einsum("bpk,pk->b", jsp, ybar_sp)
                g8 = xbar[:nq].reshape(8, q)
                for p in range(8):
                    gfl[:, nfit[i, p]] += g8[p]
                new_gV[i] = xbar[nq:nq + 3]
                new_gr[i] = xbar[nq + 3:nq + 6]
                gth += xbar[nq + 6:nq + 10]
                gfc[i] = xbar[nq + 10:nq + 13]
            if pair is not None:
                # the pair forces move with every position: columns of d F_C / d r
                for j in range(n):
                    for kk in range(3):
                        dr_ = np.zeros((n, 3), dtype=complex)
                        dr_[j, kk] = 1j * H
                        col = np.imag(pair_forces(r + dr_, shape, *pair)) / H
                        new_gr[j, kk] += (col * gfc).sum()
            gr, gV = new_gr, new_gV
        gf = gfn
    return gf, gr, gV, gth
