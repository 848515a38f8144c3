"""FP64 oracle: photo-switching operator S, acoustic operator H, A = H S, the
regulariser's proximal maps and the proximal-gradient (FISTA) solver.

TEST INFRASTRUCTURE ONLY -- see the package docstring.  Paper: arXiv
2510.23739 ("A global inverse-problem approach to quantitative
photo-switching optoacoustic mesoscopy").

Array layouts (all C-contiguous float64 unless stated):
  c   concentrations           [S][Ny][Nx][Nz]
  b   initial pressure/pulse   [K][Ny][Nx][Nz]
  y   A-scans                  [K][Ny][Nx][Nt]
  t0  band start sample        [Nz][F][F] int  (offset index jdy, jdx; dy = jdy - R)
  taps band values             [Nz][F][F][W]   (h at samples t0 .. t0+W-1)
  u   dual variable of TV      [3][S][Ny][Nx][Nz]  (differences along y, x, z)

A scan (iy, ix) sees voxel (iy + dy, ix + dx, z) through h[z][jdy][jdx][t];
voxels outside the grid and samples outside [0, Nt) do not exist.

Parity status: every function here is pinned by tests/test_oracle_*.py
against closed forms, brute force, library routines (LAPACK eigvalsh,
SciPy BVLS / NNLS) or invariants; none is "parity unpinned".
"""
from __future__ import annotations

import math
from typing import Callable, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "switching_matrix", "apply_S", "apply_ST", "band_matrix", "band_stack",
    "apply_H", "apply_HT", "apply_A", "apply_AT", "dense_A",
    "apply_A_scans", "apply_AT_columns",
    "shell_mask", "shell_matrix", "shell_stack", "apply_Lambda", "apply_LambdaT",
    "eir_conv", "eir_corr", "apply_A_fact", "apply_AT_fact", "apply_A_fact_scans",
    "apply_AT_fact_columns",
    "grad", "grad_T", "tv", "tv_step_constant", "prox_l1", "prox_tv", "prox_w",
    "switching_norm2", "r3_dual_steps", "prox_r3",
    "power_iteration", "objective", "fista", "fista_momentum", "rel_err",
]


# ----------------------------------------------------------------------------
# photo-switching operator S  (Sec. 2.2.1, eqs. final-H, Sij-detailed,
# photoswitching-full-discrete-forward-detailed)
# ----------------------------------------------------------------------------
def switching_matrix(phi, a, b, tau, gamma: float, n_pulses: int) -> np.ndarray:
    """Per-voxel switching matrix S_v[k][s].

    The deposited energy of pulse k at voxel v is the fluence times the sum
    over species of the switching extinction (eps_OFF plus the decaying ON
    part) times the concentration (eq. final-H).  With eps_OFF = a_s,
    eps_ON - eps_OFF = b_s and the rate k_p t_n written per pulse as
    Phi^gamma / tau_s (gamma = 1 is the paper's fluence-dependent rate):
        S_v[k][s] = Phi_v * (a_s + b_s * exp(-k * Phi_v**gamma / tau_s)).
    `phi` has shape [Nz] (depth profile) or [Ny][Nx][Nz]; the result has
    shape phi.shape + [K, S].
    """
    phi = np.asarray(phi, dtype=np.float64)[..., None, None]
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    tau = np.asarray(tau, dtype=np.float64)
    k = np.arange(n_pulses, dtype=np.float64)[:, None]
    rate = np.power(phi, gamma) / tau
    return phi * (a + b * np.exp(-k * rate))


def _s_at(S: np.ndarray, ny: int, nx: int) -> str:
    """einsum subscript of S: per-depth table [Nz,K,S] or per-voxel [Ny,Nx,Nz,K,S]."""
    return "zks" if S.ndim == 3 else "yxzks"


def apply_S(c: np.ndarray, S: np.ndarray) -> np.ndarray:
    """b[k][v] = sum_s S_v[k][s] c[s][v]   (block-diagonal S, one block per voxel).
    Returned C-contiguous (einsum leaves the pulse axis fastest, which sends
    every later matrix product down numpy's strided path)."""
    sub = _s_at(S, c.shape[1], c.shape[2])
    return np.ascontiguousarray(np.einsum(f"{sub},syxz->kyxz", S, np.asarray(c, dtype=np.float64)))


def apply_ST(bh: np.ndarray, S: np.ndarray) -> np.ndarray:
    """Transpose of apply_S: c[s][v] = sum_k S_v[k][s] bh[k][v] (C-contiguous)."""
    sub = _s_at(S, bh.shape[1], bh.shape[2])
    return np.ascontiguousarray(np.einsum(f"{sub},kyxz->syxz", S, np.asarray(bh, dtype=np.float64)))


# ----------------------------------------------------------------------------
# acoustic operator H  (Sec. 2.1.4 eqs. q-above-1d, q-below-1d,
# acoustic-temporal-conv; Sec. 2.2.3 eqs. acoustic-discrete-single,
# acoustic-full-forward)
# ----------------------------------------------------------------------------
def band_matrix(t0: np.ndarray, taps: np.ndarray, nt: int, jdy: int, jdx: int) -> np.ndarray:
    """Dense Nt x Nz matrix of the impulse response for one lateral offset:
    column z holds taps[z, jdy, jdx, j] at row t0[z, jdy, jdx] + j; rows
    outside [0, Nt) are dropped; everything else is zero."""
    nz, width = t0.shape[0], taps.shape[-1]
    H = np.zeros((nt, nz), dtype=np.float64)
    t = t0[:, jdy, jdx].astype(np.int64)[:, None] + np.arange(width)[None, :]
    z = np.broadcast_to(np.arange(nz)[:, None], t.shape)
    keep = (t >= 0) & (t < nt)
    H[t[keep], z[keep]] = taps[:, jdy, jdx, :].astype(np.float64)[keep]
    return H


def band_stack(t0: np.ndarray, taps: np.ndarray, nt: int) -> np.ndarray:
    """All offsets' band matrices, [F][F][Nt][Nz]."""
    f = t0.shape[1]
    return np.stack([np.stack([band_matrix(t0, taps, nt, jy, jx) for jx in range(f)])
                     for jy in range(f)])


def _overlap(n: int, d: int) -> Tuple[int, int]:
    """Scan indices i in [lo, hi) whose voxel i + d lies inside [0, n)."""
    return max(0, -d), min(n, n - d)


def apply_H(b: np.ndarray, t0: np.ndarray, taps: np.ndarray, nt: int) -> np.ndarray:
    """y[k][iy][ix][t] = sum_{dy,dx} sum_z h[z][dy][dx][t] b[k][iy+dy][ix+dx][z].

    The paper's acoustic signal of one pulse is the spatial-response-weighted
    integral of the initial pressure over the semicircle of radius |f - c0 tau|
    around the focal spot, convolved in time with the electrical impulse
    response; the banded table h holds that weight times the shifted impulse
    response for every voxel offset, so the signal is a sum over offsets of
    (Nt x Nz band) x (shifted voxel column), applied to every pulse
    independently (the block-diagonal W_tot)."""
    b = np.asarray(b, dtype=np.float64)
    K, ny, nx, nz = b.shape
    f = t0.shape[1]
    R = (f - 1) // 2
    y = np.zeros((K, ny, nx, nt), dtype=np.float64)
    for jdy in range(f):
        dy = jdy - R
        y0, y1 = _overlap(ny, dy)
        if y0 >= y1:
            continue
        for jdx in range(f):
            dx = jdx - R
            x0, x1 = _overlap(nx, dx)
            if x0 >= x1:
                continue
            H = band_matrix(t0, taps, nt, jdy, jdx)
            y[:, y0:y1, x0:x1, :] += b[:, y0 + dy:y1 + dy, x0 + dx:x1 + dx, :] @ H.T
    return y


def apply_HT(y: np.ndarray, t0: np.ndarray, taps: np.ndarray, nz: int) -> np.ndarray:
    """Adjoint of apply_H: bh[k][jy][jx][z] = sum_{dy,dx} sum_t h[z][dy][dx][t] y[k][jy-dy][jx-dx][t]."""
    y = np.asarray(y, dtype=np.float64)
    K, ny, nx, nt = y.shape
    f = t0.shape[1]
    R = (f - 1) // 2
    bh = np.zeros((K, ny, nx, nz), dtype=np.float64)
    for jdy in range(f):
        dy = jdy - R
        y0, y1 = _overlap(ny, dy)
        if y0 >= y1:
            continue
        for jdx in range(f):
            dx = jdx - R
            x0, x1 = _overlap(nx, dx)
            if x0 >= x1:
                continue
            H = band_matrix(t0, taps, nt, jdy, jdx)
            bh[:, y0 + dy:y1 + dy, x0 + dx:x1 + dx, :] += y[:, y0:y1, x0:x1, :] @ H
    return bh


def apply_A(c, S, t0, taps, nt):
    """A = W_tot S (eq. full-forward): switching per voxel, then acoustics per pulse."""
    return apply_H(apply_S(c, S), t0, taps, nt)


def apply_AT(y, S, t0, taps, nz):
    """A^T = S^T W_tot^T."""
    return apply_ST(apply_HT(y, t0, taps, nz), S)


def dense_A(shape_c: Sequence[int], n_pulses: int, nt: int, S: np.ndarray,
            t0: np.ndarray, taps: np.ndarray) -> np.ndarray:
    """Brute-force matrix of A, built entry by entry (tiny grids only):
    A[(k,iy,ix,t),(s,jy,jx,z)] = S_(jy,jx,z)[k][s] * h[z][jy-iy+R][jx-ix+R][t]
    when both lateral offsets are within the footprint."""
    n_s, ny, nx, nz = shape_c
    f = t0.shape[1]
    R = (f - 1) // 2
    width = taps.shape[-1]
    per_voxel = S.ndim == 5
    M = np.zeros((n_pulses * ny * nx * nt, n_s * ny * nx * nz))
    for k in range(n_pulses):
        for iy in range(ny):
            for ix in range(nx):
                for s in range(n_s):
                    for jy in range(ny):
                        for jx in range(nx):
                            jdy, jdx = jy - iy + R, jx - ix + R
                            if not (0 <= jdy < f and 0 <= jdx < f):
                                continue
                            for z in range(nz):
                                sv = S[jy, jx, z, k, s] if per_voxel else S[z, k, s]
                                col = ((s * ny + jy) * nx + jx) * nz + z
                                for j in range(width):
                                    t = int(t0[z, jdy, jdx]) + j
                                    if 0 <= t < nt:
                                        row = ((k * ny + iy) * nx + ix) * nt + t
                                        M[row, col] += sv * float(taps[z, jdy, jdx, j])
    return M


def _patch(arr: np.ndarray, cy: int, cx: int, R: int) -> np.ndarray:
    """arr[:, cy-R:cy+R+1, cx-R:cx+R+1, :] with zeros outside the grid."""
    n0, ny, nx, n3 = arr.shape
    out = np.zeros((n0, 2 * R + 1, 2 * R + 1, n3), dtype=np.float64)
    ya, yb = max(0, cy - R), min(ny, cy + R + 1)
    xa, xb = max(0, cx - R), min(nx, cx + R + 1)
    out[:, ya - (cy - R):yb - (cy - R), xa - (cx - R):xb - (cx - R), :] = arr[:, ya:yb, xa:xb, :]
    return out


def apply_A_scans(c, S, t0, taps, nt, scans: Sequence[Tuple[int, int]],
                  Hs: Optional[np.ndarray] = None) -> np.ndarray:
    """A c evaluated at the listed scan positions only: returns [len(scans)][K][Nt].
    Same definition as apply_A, restricted to the outputs asked for."""
    c = np.asarray(c, dtype=np.float64)
    if Hs is None:
        Hs = band_stack(t0, taps, nt)                       # [F][F][Nt][Nz]
    f = Hs.shape[0]
    R = (f - 1) // 2
    out = []
    for (iy, ix) in scans:
        cp = _patch(c, iy, ix, R)                           # [S][F][F][Nz]
        if S.ndim == 5:
            Sp = np.zeros((f, f) + S.shape[2:])
            ny, nx = c.shape[1:3]
            for jdy in range(f):
                for jdx in range(f):
                    vy, vx = iy + jdy - R, ix + jdx - R
                    if 0 <= vy < ny and 0 <= vx < nx:
                        Sp[jdy, jdx] = S[vy, vx]
            bp = np.einsum("yxzks,syxz->kyxz", Sp, cp)
        else:
            bp = np.einsum("zks,syxz->kyxz", S, cp)        # [K][F][F][Nz]
        out.append(np.einsum("yxtz,kyxz->kt", Hs, bp))
    return np.stack(out)


def apply_AT_columns(y, S, t0, taps, nz, columns: Sequence[Tuple[int, int]],
                     Hs: Optional[np.ndarray] = None) -> np.ndarray:
    """A^T y evaluated at the listed voxel columns only: returns [len][S][Nz]."""
    y = np.asarray(y, dtype=np.float64)
    nt = y.shape[3]
    if Hs is None:
        Hs = band_stack(t0, taps, nt)
    f = Hs.shape[0]
    R = (f - 1) // 2
    out = []
    for (jy, jx) in columns:
        yp = _patch(y, jy, jx, R)                           # yp[:, R+a, R+b] = y[:, jy+a, jx+b]
        # scan = voxel - offset: offset index (jdy, jdx) pairs with yp[:, F-1-jdy, F-1-jdx]
        yflip = yp[:, ::-1, ::-1, :]
        bh = np.einsum("yxtz,kyxt->kz", Hs, yflip)          # [K][Nz]
        Sv = S[jy, jx] if S.ndim == 5 else S                # [Nz][K][S]
        out.append(np.einsum("zks,kz->sz", Sv, bh))
    return np.stack(out)


# ----------------------------------------------------------------------------
# factorised acoustic operator: unit-weight discrete semicircles (shells in 3D)
# weighted by the spatial response image, then the temporal convolution with
# the electrical impulse response (Sec. 2.2.3 "Acoustic Model": eqs.
# q-above-final, q-below-final, discrete-upper-circle, discrete-lower-circle,
# acoustic-temporal-conv; App. E)
# ----------------------------------------------------------------------------
def shell_mask(nz: int, f: int, nt: int, dr: float, z_focus: float, t_focus: int) -> np.ndarray:
    """Members of the discrete shells, bool [Nt][Nz][F][F] (offset index jdy,
    jdx as in the banded table).

    Sample t is the sphere of radius rho_t = |t - t_focus| dr (in voxel
    pitches) around the focal point: its upper half (voxels whose centre lies
    above the focal plane, z < z_focus) for t < t_focus and its lower half
    (centre depth >= z_focus) for t >= t_focus.  A voxel belongs to the
    shell when its box (one pitch wide around its centre) meets the sphere:
    the box's nearest point is at distance <= rho_t and its farthest at
    distance >= rho_t.  The paper keeps every pixel the semicircle crosses
    with unit weight instead of its arc length; this is the same rule with
    voxels and spheres.  Squared distances are summed in the order y, x, z."""
    R = (f - 1) // 2
    off = np.arange(-R, R + 1, dtype=np.float64)
    dz = np.arange(nz, dtype=np.float64) - z_focus
    near = lambda o: np.maximum(np.abs(o) - 0.5, 0.0)   # nearest box coordinate
    far = lambda o: np.abs(o) + 0.5                     # farthest box coordinate
    lat_near = near(off)[:, None] * near(off)[:, None] + near(off)[None, :] * near(off)[None, :]
    lat_far = far(off)[:, None] * far(off)[:, None] + far(off)[None, :] * far(off)[None, :]
    dmin2 = lat_near[None] + (near(dz) * near(dz))[:, None, None]      # [Nz][F][F]
    dmax2 = lat_far[None] + (far(dz) * far(dz))[:, None, None]
    below = np.broadcast_to((dz >= 0.0)[:, None, None], dmin2.shape)
    t = np.arange(nt, dtype=np.int64)
    rho = np.abs(t - int(t_focus)).astype(np.float64) * dr
    rho2 = (rho * rho)[:, None, None, None]
    lower = (t >= t_focus)[:, None, None, None]
    side = np.where(lower, below[None], ~below[None])
    return side & (dmin2[None] <= rho2) & (rho2 <= dmax2[None])


def shell_matrix(spr: np.ndarray, mask: np.ndarray, jdy: int, jdx: int) -> np.ndarray:
    """Nt x Nz matrix of one lateral offset: eta[z][jdy][jdx] where voxel z is
    in shell t, zero elsewhere."""
    return mask[:, :, jdy, jdx] * np.asarray(spr, dtype=np.float64)[None, :, jdy, jdx]


def shell_stack(spr: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """All offsets' shell matrices, [F][F][Nt][Nz]."""
    f = spr.shape[1]
    return np.stack([np.stack([shell_matrix(spr, mask, jy, jx) for jx in range(f)])
                     for jy in range(f)])


def apply_Lambda(b: np.ndarray, spr: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """Spatial integration of every pulse: q[k][iy][ix][t] = sum over the voxels
    (iy + dy, ix + dx, z) of shell t of eta[z][dy][dx] b[k][iy+dy][ix+dx][z]
    (the product of the initial pressure with the spatial response shifted to
    the scan position, summed over the discrete semicircle).  Voxels outside
    the grid do not exist."""
    b = np.asarray(b, dtype=np.float64)
    K, ny, nx, nz = b.shape
    nt, f = mask.shape[0], mask.shape[2]
    R = (f - 1) // 2
    q = np.zeros((K, ny, nx, nt), dtype=np.float64)
    for jdy in range(f):
        dy = jdy - R
        y0, y1 = _overlap(ny, dy)
        if y0 >= y1:
            continue
        for jdx in range(f):
            dx = jdx - R
            x0, x1 = _overlap(nx, dx)
            if x0 >= x1:
                continue
            L = shell_matrix(spr, mask, jdy, jdx)
            q[:, y0:y1, x0:x1, :] += b[:, y0 + dy:y1 + dy, x0 + dx:x1 + dx, :] @ L.T
    return q


def apply_LambdaT(q: np.ndarray, spr: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """Adjoint of apply_Lambda."""
    q = np.asarray(q, dtype=np.float64)
    K, ny, nx, nt = q.shape
    nz, f = mask.shape[1], mask.shape[2]
    R = (f - 1) // 2
    b = np.zeros((K, ny, nx, nz), dtype=np.float64)
    for jdy in range(f):
        dy = jdy - R
        y0, y1 = _overlap(ny, dy)
        if y0 >= y1:
            continue
        for jdx in range(f):
            dx = jdx - R
            x0, x1 = _overlap(nx, dx)
            if x0 >= x1:
                continue
            L = shell_matrix(spr, mask, jdy, jdx)
            b[:, y0 + dy:y1 + dy, x0 + dx:x1 + dx, :] += q[:, y0:y1, x0:x1, :] @ L
    return b


def eir_conv(q: np.ndarray, v: np.ndarray, origin: int) -> np.ndarray:
    """Temporal convolution of every A-scan with the electrical impulse
    response: p[t] = sum_j v[j] q[t - j + origin] (v[origin] is the zero-lag
    tap); samples outside [0, Nt) are zero."""
    q = np.asarray(q, dtype=np.float64)
    nt = q.shape[-1]
    p = np.zeros_like(q)
    for j, vj in enumerate(np.asarray(v, dtype=np.float64)):
        lag = j - origin
        if abs(lag) >= nt:
            continue
        if lag >= 0:
            p[..., lag:] += vj * q[..., :nt - lag]
        else:
            p[..., :nt + lag] += vj * q[..., -lag:]
    return p


def eir_corr(r: np.ndarray, v: np.ndarray, origin: int) -> np.ndarray:
    """Adjoint of eir_conv: u[t] = sum_j v[j] r[t + j - origin]."""
    r = np.asarray(r, dtype=np.float64)
    nt = r.shape[-1]
    u = np.zeros_like(r)
    for j, vj in enumerate(np.asarray(v, dtype=np.float64)):
        lag = j - origin
        if abs(lag) >= nt:
            continue
        if lag >= 0:
            u[..., :nt - lag] += vj * r[..., lag:]
        else:
            u[..., -lag:] += vj * r[..., :nt + lag]
    return u


def apply_A_fact(c, S, spr, mask, v, origin):
    """A = V Lambda S: switching, spatial integration over the shells, then the
    temporal convolution (eq. full-forward with the factorised W)."""
    return eir_conv(apply_Lambda(apply_S(c, S), spr, mask), v, origin)


def apply_AT_fact(y, S, spr, mask, v, origin):
    """A^T = S^T Lambda^T V^T."""
    return apply_ST(apply_LambdaT(eir_corr(y, v, origin), spr, mask), S)


def apply_A_fact_scans(c, S, spr, mask, v, origin, scans, Ls=None):
    """apply_A_fact at the listed scan positions only: [len(scans)][K][Nt]."""
    if Ls is None:
        Ls = shell_stack(spr, mask)
    q = apply_A_scans(c, S, None, None, mask.shape[0], scans, Hs=Ls)
    return eir_conv(q, v, origin)


def apply_AT_fact_columns(y, S, spr, mask, v, origin, columns, Ls=None):
    """apply_AT_fact at the listed voxel columns only: [len(columns)][S][Nz]."""
    if Ls is None:
        Ls = shell_stack(spr, mask)
    return apply_AT_columns(eir_corr(y, v, origin), S, None, None, mask.shape[1], columns, Hs=Ls)


# ----------------------------------------------------------------------------
# regulariser: anisotropic TV, l1, nonnegativity  (eqs. reg-tv-l1-one, prox,
# prox-dual; Alg. "alg:prox-inner")
# ----------------------------------------------------------------------------
def grad(x: np.ndarray) -> np.ndarray:
    """Forward differences along y, x and z of every species volume, Neumann
    boundary (the last difference along each axis is 0): [3] + x.shape."""
    x = np.asarray(x, dtype=np.float64)
    g = np.zeros((3,) + x.shape, dtype=np.float64)
    for d, ax in enumerate((-3, -2, -1)):
        n = x.shape[ax]
        hi = [slice(None)] * x.ndim
        lo = [slice(None)] * x.ndim
        hi[ax] = slice(1, n)
        lo[ax] = slice(0, n - 1)
        g[d][tuple(lo)] = x[tuple(hi)] - x[tuple(lo)]
    return g


def grad_T(p: np.ndarray) -> np.ndarray:
    """Exact adjoint of grad (minus the divergence)."""
    p = np.asarray(p, dtype=np.float64)
    out = np.zeros(p.shape[1:], dtype=np.float64)
    for d, ax in enumerate((-3, -2, -1)):
        n = out.shape[ax]
        hi = [slice(None)] * out.ndim
        lo = [slice(None)] * out.ndim
        hi[ax] = slice(1, n)
        lo[ax] = slice(0, n - 1)
        out[tuple(lo)] -= p[d][tuple(lo)]
        out[tuple(hi)] += p[d][tuple(lo)]
    return out


def tv(x: np.ndarray) -> float:
    """Anisotropic TV summed over species: sum of |differences| along y, x, z."""
    return float(np.abs(grad(x)).sum())


def tv_step_constant(shape_v: Sequence[int]) -> float:
    """Largest eigenvalue of grad^T grad on one volume: the path-graph Laplacian
    on n nodes has largest eigenvalue 4 sin^2(pi (n-1) / (2n)), and the 3D
    operator is their Kronecker sum.  The dual step is its reciprocal
    (alpha_2 = 1/eig_max(L L^T) in Alg. alg:prox-inner)."""
    return float(sum(4.0 * math.sin(math.pi * (n - 1) / (2.0 * n)) ** 2 for n in shape_v))


def prox_l1(z: np.ndarray, thresh: float, nonneg: bool = True) -> np.ndarray:
    """Proximal map of thresh*||.||_1 (+ indicator of x >= 0 when nonneg):
    soft threshold sign(z) max(|z| - thresh, 0), or max(z - thresh, 0)."""
    z = np.asarray(z, dtype=np.float64)
    if nonneg:
        return np.maximum(z - thresh, 0.0)
    return np.sign(z) * np.maximum(np.abs(z) - thresh, 0.0)


def fista_momentum(t: float, literal: bool = False) -> Tuple[float, float]:
    """Next FISTA step t' = (1 + sqrt(1 + 4 t^2)) / 2 and the extrapolation
    weight: (t - 1)/t' (Beck-Teboulle), or the printed (t - 1)/(t + 1)."""
    t_next = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * t * t))
    beta = (t - 1.0) / (t + 1.0) if literal else (t - 1.0) / t_next
    return t_next, beta


def prox_tv(z: np.ndarray, theta: float, n_inner: int, nonneg: bool = False,
            u_init: Optional[np.ndarray] = None, literal_momentum: bool = False,
            return_dual: bool = False):
    """Proximal map of theta*TV by accelerated projected gradient on the dual
    (Alg. alg:prox-inner with L = grad, eq. prox-dual):
        u_{j+1} = clip(eta_j + (1/mu) grad(z - grad^T eta_j), -theta, theta)
        eta_{j+1} = u_{j+1} + beta_j (u_{j+1} - u_j)
    starting from u_0 = eta_0 = 0 (or u_init), exactly n_inner steps, then
    x = z - grad^T u (clamped at 0 when nonneg, the algorithm's output step).
    Writing the dual of L = lambda*grad as u = lambda*u' turns the printed
    projection radius alpha_1 into theta = alpha_1 * lambda."""
    z = np.asarray(z, dtype=np.float64)
    mu = tv_step_constant(z.shape[-3:])
    u = np.zeros((3,) + z.shape) if u_init is None else np.array(u_init, dtype=np.float64)
    eta = u.copy()
    t = 1.0
    for _ in range(n_inner):
        u_next = np.clip(eta + grad(z - grad_T(eta)) / mu, -theta, theta)
        t, beta = fista_momentum(t, literal_momentum)
        eta = u_next + beta * (u_next - u)
        u = u_next
    x = z - grad_T(u)
    if nonneg:
        x = np.maximum(x, 0.0)
    return (x, u) if return_dual else x


def prox_w(z: np.ndarray, theta_tv: float, theta_l1: float, n_inner: int,
           literal_momentum: bool = False) -> np.ndarray:
    """Proximal map of theta_tv*TV + theta_l1*||.||_1 + indicator(x >= 0)
    (the one-step regulariser without the TV(Sc) term, eqs. one-step,
    reg-tv-l1-one, prox).  TV is a sum of |x_i - x_j| over graph edges and
    the other two terms are the same monotone separable function on every
    coordinate, so the map is soft-thresholding-with-clamp applied after the
    TV prox; the clamp is the algorithm's final max(., 0)."""
    x = prox_tv(z, theta_tv, n_inner, nonneg=False, literal_momentum=literal_momentum)
    return np.maximum(x - theta_l1, 0.0)


# ----------------------------------------------------------------------------
# the full one-step regulariser R3 with its TV(S c) term  (eq. reg-tv-l1-one;
# the stacked operator L = [L1; L2; L3] and Alg. alg:prox-inner on its dual)
# ----------------------------------------------------------------------------
def switching_norm2(S: np.ndarray) -> float:
    """max over voxels of the squared spectral norm of S_v ([K][S] blocks)."""
    S = np.asarray(S, dtype=np.float64)
    return float(np.max(np.linalg.norm(S, ord=2, axis=(-2, -1)) ** 2))


def r3_dual_steps(shape_v: Sequence[int], S: np.ndarray, theta_tv: float, theta_tvs: float,
                  theta_l1: float) -> Tuple[float, float, float]:
    """Per-block dual steps of the stacked prox.  With L = [l1 grad; l2 grad S;
    l3 I] and the duals rescaled block by block (u_b = l_b u'_b, so the
    projection radius alpha_1 of Alg. alg:prox-inner becomes theta_b =
    alpha_1 l_b), the step alpha_2 = 1/eig_max(L^T L) multiplies block b by
    l_b^2, i.e. theta_b^2 / (sum_b' theta_b'^2 m_b').  eig_max(L^T L) is
    replaced by the upper bound sum_b l_b^2 m_b with m_1 = eig_max(grad^T grad)
    (closed form), m_2 = m_1 * max_v |S_v|^2 (|grad S x| <= |grad| |S x|) and
    m_3 = 1: the eigenvalues of a sum of symmetric PSD matrices are at most the
    sum of their largest ones, so the step stays at or below 1/eig_max."""
    mu = tv_step_constant(shape_v)
    bsum = theta_tv ** 2 * mu + theta_tvs ** 2 * mu * switching_norm2(S) + theta_l1 ** 2
    if bsum == 0.0:
        return 0.0, 0.0, 0.0
    return theta_tv ** 2 / bsum, theta_tvs ** 2 / bsum, theta_l1 ** 2 / bsum


def prox_r3(z: np.ndarray, S: np.ndarray, theta_tv: float, theta_tvs: float, theta_l1: float,
            n_inner: int, literal_momentum: bool = False, return_dual: bool = False):
    """Proximal map of theta_tv TV(x) + theta_tvs sum_k TV((S x)^k) +
    theta_l1 |x|_1 + indicator(x >= 0) by the paper's dual iteration on the
    stacked operator (Alg. alg:prox-inner, eq. prox-dual, L of eq.
    reg-tv-l1-one's text: TV of c, TV of S c, l1):
        w = z - (grad^T e1 + S^T grad^T e2 + e3)
        u1' = clip(e1 + s1 grad w, theta_tv)
        u2' = clip(e2 + s2 grad (S w), theta_tvs)
        u3' = clip(e3 + s3 w, theta_l1)
        e_b = u_b' + beta (u_b' - u_b)
    from zero duals, exactly n_inner steps (steps s_b from r3_dual_steps),
    then x = max(z - (grad^T u1 + S^T grad^T u2 + u3), 0).
    The iteration projects the duals onto their boxes only and clamps at the
    end, as printed; it converges to the clamp of the prox of the regulariser
    without the sign constraint, which equals the prox with it when
    theta_tvs = 0 or S does not mix species, and differs otherwise.
    z: [S][Ny][Nx][Nz]; S: [Nz][K][S] or [Ny][Nx][Nz][K][S]."""
    z = np.asarray(z, dtype=np.float64)
    s1, s2, s3 = r3_dual_steps(z.shape[-3:], S, theta_tv, theta_tvs, theta_l1)
    n_k = S.shape[-2]
    u1 = np.zeros((3,) + z.shape)
    u2 = np.zeros((3, n_k) + z.shape[1:])
    u3 = np.zeros(z.shape)
    e1, e2, e3 = u1.copy(), u2.copy(), u3.copy()
    t = 1.0

    def lt(a1, a2, a3):
        return grad_T(a1) + apply_ST(grad_T(a2), S) + a3

    for _ in range(n_inner):
        w = z - lt(e1, e2, e3)
        n1 = np.clip(e1 + s1 * grad(w), -theta_tv, theta_tv)
        n2 = np.clip(e2 + s2 * grad(apply_S(w, S)), -theta_tvs, theta_tvs)
        n3 = np.clip(e3 + s3 * w, -theta_l1, theta_l1)
        t, beta = fista_momentum(t, literal_momentum)
        e1, e2, e3 = n1 + beta * (n1 - u1), n2 + beta * (n2 - u2), n3 + beta * (n3 - u3)
        u1, u2, u3 = n1, n2, n3
    x = np.maximum(z - lt(u1, u2, u3), 0.0)
    return (x, (u1, u2, u3)) if return_dual else x


# ----------------------------------------------------------------------------
# solver  (Alg. alg:prox-outer; eq. one-step)
# ----------------------------------------------------------------------------
def power_iteration(A: Callable, AT: Callable, v0: np.ndarray, n_iter: int) -> float:
    """Estimate eig_max(A^T A) (the step alpha_1 = 1/eig_max is set in
    Alg. alg:prox-outer; the paper does not say how it is computed):
    v <- v0/|v0|; repeat n_iter times { w = A^T A v; lam = <v, w>; v = w/|w| }."""
    v = np.asarray(v0, dtype=np.float64)
    v = v / np.linalg.norm(v)
    lam = 0.0
    for _ in range(n_iter):
        w = AT(A(v))
        lam = float(np.vdot(v, w))
        v = w / np.linalg.norm(w)
    return lam


def objective(c, p, A: Callable, lam_tv: float, lam_l1: float, lam_tvs: float = 0.0,
              S: Optional[np.ndarray] = None) -> float:
    """F(c) = 1/2 |A c - p|^2 + lam_tv TV(c) + lam_l1 |c|_1 + lam_tvs TV(S c)
    (eq. one-step with R3 of eq. reg-tv-l1-one; c is assumed nonnegative)."""
    r = A(c) - p
    f = 0.5 * float(np.vdot(r, r)) + lam_tv * tv(c) + lam_l1 * float(np.abs(c).sum())
    if lam_tvs > 0.0:
        f += lam_tvs * tv(apply_S(c, S))
    return f


def fista(p, A: Callable, AT: Callable, alpha1: float, lam_tv: float, lam_l1: float,
          k1: int, k2: int, c_init=None, eps1: float = 0.0, eps2: float = 0.0,
          literal_momentum: bool = False, momentum: bool = True,
          trace: Optional[list] = None, shape_c=None, lam_tvs: float = 0.0,
          S: Optional[np.ndarray] = None):
    """Proximal gradient with FISTA momentum (Alg. alg:prox-outer):
        c_{k+1} = prox_{alpha1 w}(xi_k - alpha1 A^T (A xi_k - p))
        t_{k+1} = (1 + sqrt(1 + 4 t_k^2))/2
        xi_{k+1} = c_{k+1} + beta_k (c_{k+1} - c_k)
    from c_0 = xi_0 = 0 (or c_init), exactly k1 iterations unless a stopping
    test fires (relative objective change < eps1 or relative xi change < eps2,
    checked from the third iteration on; a zero eps disables its test).
    The gradient is formed as A^T (A xi - p), equal to the printed
    A^T A xi - A^T p.  momentum=False gives plain proximal gradient (ISTA).
    With lam_tvs > 0 (the TV(S c) term, S given) the prox is the stacked dual
    iteration prox_r3; otherwise the exact composition prox_w.
    Returns (c_final, iterations)."""
    if c_init is None:
        c = np.zeros(shape_c, dtype=np.float64)
    else:
        c = np.array(c_init, dtype=np.float64)
    xi = c.copy()
    t = 1.0
    f_prev = None
    it = 0
    for k in range(k1):
        g = AT(A(xi) - p)
        if lam_tvs > 0.0:
            c_next = prox_r3(xi - alpha1 * g, S, alpha1 * lam_tv, alpha1 * lam_tvs,
                             alpha1 * lam_l1, k2, literal_momentum)
        else:
            c_next = prox_w(xi - alpha1 * g, alpha1 * lam_tv, alpha1 * lam_l1, k2, literal_momentum)
        t, beta = fista_momentum(t, literal_momentum)
        if not momentum:
            beta = 0.0
        xi_next = c_next + beta * (c_next - c)
        it = k + 1
        stop = False
        f_now = None
        if eps1 > 0.0 or trace is not None:
            f_now = objective(c_next, p, A, lam_tv, lam_l1, lam_tvs, S)
            if trace is not None:
                trace.append(f_now)
        if k > 1:
            if eps1 > 0.0 and f_prev is not None and abs(f_now - f_prev) < eps1 * abs(f_prev):
                stop = True
            nx = np.linalg.norm(xi)
            if eps2 > 0.0 and nx > 0.0 and np.linalg.norm(xi_next - xi) < eps2 * nx:
                stop = True
        f_prev = f_now
        c, xi = c_next, xi_next
        if stop:
            break
    return c, it


def rel_err(x, ref) -> float:
    """Normwise relative error |x - ref|_2 / |ref|_2 (the paper's NRMSE, App. B)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    n = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / n) if n > 0 else float(np.linalg.norm(x))
