"""FP64 reverse-mode reference for the gradients of the coupled step
(TEST INFRASTRUCTURE ONLY: the tests are its only callers; it shares no code
with the HIP library, the C oracle or the brute-force stepper).

A third, separately written implementation of the discrete scheme of
arXiv:2510.22221, Methods, "Numerical Model", on small boxes with PEC walls:
CPU torch tensors in float64 over the natural Yee arrays, so that torch's
reverse-mode automatic differentiation gives the exact gradients of a loss of
the run with respect to the bias field H0, the permittivity of chosen cells
and the saturation magnetisation of chosen cells.

One full step (the half-step reading of the dt/4 and dt/(2 mu0) factors):
  * H/M half step of length dt/2 with E^n: at every face B^ = H + M_c and
    B^* = B^ - dt/(2 mu0) (curl E)_c (eq. iterate_H with B = mu0 (H + M));
    non-magnetic faces take H = B^*; at a magnetic face the trapezoidal LLG
    update (eqs. llg_tra4-llg_tra6) is solved in closed form,
      a = -(k P + (alpha/Ms) M),  b = M - k M x Q,  k = mu0 |gamma| dt / 4,
      X = (b + (a.b) a - a x b) / (1 + |a|^2),  M' = Ms X / |X|,
    with P and Q the field at the face from B^* and B^ (normal component: the
    face's own; transverse ones: the mean of the nearest faces of that
    family) plus H0, and then H = B^*_c - M'_c;
  * E step: E <- ca E + cb ((curl H) - J) on every edge that is not PEC,
    ca = (eps/dt - sigma/2) / (eps/dt + sigma/2), cb = 1 / (eps/dt + sigma/2),
    eps and sigma the means over the cells that share the edge;
  * H/M half step with E^{n+1}.
Sites: Ex[k, j, i] at ((i+1/2) dx, j dy, k dz), Ey at (i dx, (j+1/2) dy,
k dz), Ez at (i dx, j dy, (k+1/2) dz); Hx at (i dx, (j+1/2) dy, (k+1/2) dz),
Hy at ((i+1/2) dx, j dy, (k+1/2) dz), Hz at ((i+1/2) dx, (j+1/2) dy, k dz).
A face's Ms is the mean over the (one or two) cells beside it, its alpha and
|gamma| the means over the magnetic ones among them; M starts as Ms u/|u|.
"""
from __future__ import annotations

import math

import numpy as np
import torch

MU0 = 4e-7 * math.pi
C0 = 299792458.0
EPS0 = 1.0 / (MU0 * C0 * C0)
F64 = torch.float64


def _e_shape(c, n):
    nx, ny, nz = n
    return [(nz + 1, ny + 1, nx), (nz + 1, ny, nx + 1), (nz, ny + 1, nx + 1)][c]


def _h_shape(c, n):
    nx, ny, nz = n
    return [(nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)][c]


class Reverse:
    """The scheme on a PEC box.  Parameters with gradients:
    `H0` (3,), `eps_patch` over eps_box and `ms_patch` over ms_box (numpy
    order [k, j, i]; each cell of the box its own parameter)."""

    def __init__(self, w, eps_box=(0, 0, 0, 0, 0, 0), ms_box=(0, 0, 0, 0, 0, 0)):
        if any(b != 0 for b in w.bc):
            raise ValueError("the reverse-mode reference takes PEC boxes only")
        self.n = (w.nx, w.ny, w.nz)
        self.d = tuple(float(v) for v in w.d)
        self.dt = float(w.dt)
        nx, ny, nz = self.n
        tab = np.asarray(w.materials, dtype=np.float64)
        ids = np.asarray(w.ids)
        self.H0 = torch.tensor(w.H0, dtype=F64, requires_grad=True)
        i0, j0, k0, ni, nj, nk = eps_box
        self.eps_box, self.ms_box = tuple(eps_box), tuple(ms_box)
        self._eps_host = tab[ids, 0]
        self._ms_host = tab[ids, 3]
        self.eps_patch = torch.tensor(self._eps_host[k0:k0 + nk, j0:j0 + nj, i0:i0 + ni], dtype=F64,
                                      requires_grad=True)
        i1, j1, k1, mi, mj, mk = ms_box
        self.ms_patch = torch.tensor(self._ms_host[k1:k1 + mk, j1:j1 + mj, i1:i1 + mi], dtype=F64,
                                     requires_grad=True)
        self.sig = torch.tensor(tab[ids, 1], dtype=F64)
        self.pec = tab[ids, 2] != 0
        self.magnetic = tab[ids, 3] > 0
        self.alpha = tab[ids, 4]
        self.gamma = tab[ids, 5]
        self.ids = ids
        self.mdir = np.asarray(w.m_dir, dtype=np.float64)
        self.sources = [(s.comp, s.box, np.asarray(s.table, dtype=np.float64)) for s in w.sources]

    # ----------------------------------------------------------------- cells
    def _cell_eps(self):
        i0, j0, k0, ni, nj, nk = self.eps_box
        eps = torch.tensor(self._eps_host, dtype=F64)
        if ni * nj * nk:
            eps[k0:k0 + nk, j0:j0 + nj, i0:i0 + ni] = self.eps_patch
        return eps

    def _cell_ms(self):
        i1, j1, k1, mi, mj, mk = self.ms_box
        ms = torch.tensor(self._ms_host, dtype=F64)
        if mi * mj * mk:
            ms[k1:k1 + mk, j1:j1 + mj, i1:i1 + mi] = self.ms_patch
        return ms

    # ----------------------------------------------------------------- set-up
    def _edge_coefs(self, eps_cell):
        """ca, cb on the edges of each family (zero on PEC and wall edges)."""
        nx, ny, nz = self.n
        sig = self.sig
        out = []
        for c in range(3):
            shp = _e_shape(c, self.n)
            # the cells sharing an edge: offsets -1 and 0 along the two other axes
            a1, a2 = [a for a in range(3) if a != c]
            se = torch.zeros(shp, dtype=F64)
            ss = torch.zeros(shp, dtype=F64)
            cnt = np.zeros(shp)
            anypec = np.zeros(shp, dtype=bool)
            for u in (-1, 0):
                for v in (-1, 0):
                    off = [0, 0, 0]
                    off[a1], off[a2] = u, v
                    # cell index (i, j, k) = edge index + off along a1, a2
                    sl_e, sl_c = [], []
                    for ax_np, ax in ((0, 2), (1, 1), (2, 0)):   # numpy axis -> grid axis
                        nax = self.n[ax]
                        lo_e = max(0, -off[ax])
                        hi_e = min(shp[ax_np], nax - off[ax])
                        sl_e.append(slice(lo_e, hi_e))
                        sl_c.append(slice(lo_e + off[ax], hi_e + off[ax]))
                    sl_e, sl_c = tuple(sl_e), tuple(sl_c)
                    se[sl_e] = se[sl_e] + eps_cell[sl_c]
                    ss[sl_e] = ss[sl_e] + sig[sl_c]
                    cnt[sl_e] += 1
                    anypec[sl_e] |= self.pec[sl_c]
            wall = np.zeros(shp, dtype=bool)
            for ax_np, ax in ((0, 2), (1, 1), (2, 0)):
                if ax == c:
                    continue
                idx = [slice(None)] * 3
                idx[ax_np] = 0
                wall[tuple(idx)] = True
                idx[ax_np] = shp[ax_np] - 1
                wall[tuple(idx)] = True
            live = torch.tensor(~(wall | anypec))
            cnt_t = torch.tensor(np.maximum(cnt, 1), dtype=F64)
            e = EPS0 * se / cnt_t
            s_ = ss / cnt_t
            den = e / self.dt + s_ / 2
            ca = torch.where(live, (e / self.dt - s_ / 2) / den, torch.zeros_like(den))
            cb = torch.where(live, 1.0 / den, torch.zeros_like(den))
            out.append((ca, cb))
        return out

    def _face_params(self, ms_cell):
        """Per family: flat indices of the magnetic faces, their Ms (a
        function of the Ms parameters), alpha and |gamma|."""
        out = []
        for c in range(3):
            shp = _h_shape(c, self.n)
            ax_np = 2 - c
            cells_ms = []
            cells_mag = []
            cells_al = []
            cells_ga = []
            valid = []
            for side in (-1, 0):
                # cell index along axis c = face index + side
                sl_f, sl_c = [slice(None)] * 3, [slice(None)] * 3
                lo = max(0, -side)
                hi = min(shp[ax_np], self.n[c] - side)
                sl_f[ax_np] = slice(lo, hi)
                sl_c[ax_np] = slice(lo + side, hi + side)
                m = torch.zeros(shp, dtype=F64)
                m[tuple(sl_f)] = ms_cell[tuple(sl_c)]
                g = np.zeros(shp, dtype=bool)
                g[tuple(sl_f)] = self.magnetic[tuple(sl_c)]
                a = np.zeros(shp)
                a[tuple(sl_f)] = self.alpha[tuple(sl_c)]
                y = np.zeros(shp)
                y[tuple(sl_f)] = self.gamma[tuple(sl_c)]
                v = np.zeros(shp, dtype=bool)
                v[tuple(sl_f)] = True
                cells_ms.append(m)
                cells_mag.append(g)
                cells_al.append(a)
                cells_ga.append(y)
                valid.append(v)
            nval = valid[0].astype(float) + valid[1].astype(float)
            ms_face = (cells_ms[0] + cells_ms[1]) / torch.tensor(np.maximum(nval, 1), dtype=F64)
            nmag = cells_mag[0].astype(float) + cells_mag[1].astype(float)
            mag = nmag > 0
            al = np.where(mag, (cells_al[0] * cells_mag[0] + cells_al[1] * cells_mag[1]) / np.maximum(nmag, 1), 0)
            ga = np.where(mag, (cells_ga[0] * cells_mag[0] + cells_ga[1] * cells_mag[1]) / np.maximum(nmag, 1), 0)
            flat = np.nonzero(mag.ravel())[0]
            out.append({"idx": torch.tensor(flat), "ms": ms_face.reshape(-1)[flat],
                        "al": torch.tensor(al.ravel()[flat], dtype=F64),
                        "ga": torch.tensor(ga.ravel()[flat], dtype=F64), "shape": shp})
        return out

    def _transverse_index(self, c, cp, flat):
        """Flat indices (into family cp's array) of the four faces of family
        cp nearest to each family-c face in `flat` (offsets -1/2, +1/2 along
        c and cp), and the count present (a face beside the domain's edge has
        fewer)."""
        shp_c, shp_p = _h_shape(c, self.n), _h_shape(cp, self.n)
        kk, jj, ii = np.unravel_index(flat.numpy(), shp_c)
        pos = {0: ii, 1: jj, 2: kk}
        lists, present = [], []
        for u in (-1, 0):
            for v in (-1, 0):
                # along c the cp-face sits half a cell off: index + u (+1 for
                # the +1/2 side) -- the family-c face is at an integer
                # position along c and the cp faces at half-integer ones
                q = {a: pos[a].copy() for a in range(3)}
                q[c] = pos[c] + u
                q[cp] = pos[cp] + 1 + v
                ok = np.ones_like(ii, dtype=bool)
                for a, npax in ((0, 2), (1, 1), (2, 0)):
                    ok &= (q[a] >= 0) & (q[a] < shp_p[npax])
                fl = np.ravel_multi_index((np.clip(q[2], 0, shp_p[0] - 1), np.clip(q[1], 0, shp_p[1] - 1),
                                           np.clip(q[0], 0, shp_p[2] - 1)), shp_p)
                lists.append(torch.tensor(fl))
                present.append(ok)
        return lists, [torch.tensor(p.astype(float), dtype=F64) for p in present]

    # ----------------------------------------------------------------- curls
    def _curl_e(self, E):
        dx, dy, dz = self.d
        Ex, Ey, Ez = E
        # Hx: dEz/dy - dEy/dz ; Hy: dEx/dz - dEz/dx ; Hz: dEy/dx - dEx/dy
        cx = (Ez[:, 1:, :] - Ez[:, :-1, :]) / dy - (Ey[1:, :, :] - Ey[:-1, :, :]) / dz
        cy = (Ex[1:, :, :] - Ex[:-1, :, :]) / dz - (Ez[:, :, 1:] - Ez[:, :, :-1]) / dx
        cz = (Ey[:, :, 1:] - Ey[:, :, :-1]) / dx - (Ex[:, 1:, :] - Ex[:, :-1, :]) / dy
        return cx, cy, cz

    def _curl_h(self, H):
        dx, dy, dz = self.d
        Hx, Hy, Hz = H
        pad = torch.nn.functional.pad
        # Ex: dHz/dy - dHy/dz on interior edges (wall edges are never updated)
        cx = pad((Hz[:, 1:, :] - Hz[:, :-1, :]) / dy, (0, 0, 1, 1, 0, 0))[:, :, :] \
            - pad((Hy[1:, :, :] - Hy[:-1, :, :]) / dz, (0, 0, 0, 0, 1, 1))
        cy = pad((Hx[1:, :, :] - Hx[:-1, :, :]) / dz, (0, 0, 0, 0, 1, 1)) \
            - pad((Hz[:, :, 1:] - Hz[:, :, :-1]) / dx, (1, 1, 0, 0, 0, 0))
        cz = pad((Hy[:, :, 1:] - Hy[:, :, :-1]) / dx, (1, 1, 0, 0, 0, 0)) \
            - pad((Hx[:, 1:, :] - Hx[:, :-1, :]) / dy, (0, 0, 1, 1, 0, 0))
        return cx, cy, cz

    # ----------------------------------------------------------------- run
    def run(self, nsteps, loss="film_energy", loss_from=0, film_cells=None, field=0, ijk=(0, 0, 0),
            weights=None):
        """Steps nsteps from rest and returns the loss as a torch scalar:
        "film_energy": dt * sum over n = loss_from+1 .. nsteps of the EM
        energy in `film_cells` (an [nz, ny, nx] bool mask) at integer time n;
        "trace": sum_i weights[i] E_field(ijk) after step i+1."""
        eps_cell = self._cell_eps()
        ms_cell = self._cell_ms()
        coefs = self._edge_coefs(eps_cell)
        faces = self._face_params(ms_cell)
        trans = {}
        for c in range(3):
            for cp in range(3):
                if cp != c:
                    trans[(c, cp)] = self._transverse_index(c, cp, faces[c]["idx"])
        u = self.mdir / np.linalg.norm(self.mdir)
        # M on the magnetic faces of each family: [nsite, 3]
        M = [f["ms"][:, None] * torch.tensor(u, dtype=F64)[None, :] for f in faces]
        E = [torch.zeros(_e_shape(c, self.n), dtype=F64) for c in range(3)]
        H = [torch.zeros(_h_shape(c, self.n), dtype=F64) for c in range(3)]
        k0 = MU0 * self.dt / 4.0
        hc = self.dt / (2.0 * MU0)
        H0 = self.H0

        def half(E, H, M):
            curl = self._curl_e(E)
            bn, bs = [], []
            for c in range(3):
                b = H[c].reshape(-1)
                if faces[c]["idx"].numel():
                    b = b.index_add(0, faces[c]["idx"], M[c][:, c])
                bn.append(b)
                bs.append(b - hc * curl[c].reshape(-1))
            newH, newM = [], []
            for c in range(3):
                F = faces[c]
                if F["idx"].numel() == 0:
                    newH.append(bs[c].reshape(H[c].shape))
                    newM.append(M[c])
                    continue
                Pc, Qc = [None] * 3, [None] * 3
                Pc[c] = bs[c][F["idx"]]
                Qc[c] = bn[c][F["idx"]]
                for cp in range(3):
                    if cp == c:
                        continue
                    lists, present = trans[(c, cp)]
                    cnt = sum(present)
                    Pc[cp] = sum(bs[cp][l] * p for l, p in zip(lists, present)) / cnt
                    Qc[cp] = sum(bn[cp][l] * p for l, p in zip(lists, present)) / cnt
                P = torch.stack(Pc, 1) + H0[None, :]
                Q = torch.stack(Qc, 1) + H0[None, :]
                Mo = M[c]
                kk = (k0 * F["ga"])[:, None]
                a = -(kk * P + (F["al"] / F["ms"])[:, None] * Mo)
                b = Mo - kk * torch.linalg.cross(Mo, Q, dim=1)
                ab = (a * b).sum(1, keepdim=True)
                aa = (a * a).sum(1, keepdim=True)
                X = (b + ab * a - torch.linalg.cross(a, b, dim=1)) / (1.0 + aa)
                Mn = F["ms"][:, None] * X / torch.sqrt((X * X).sum(1, keepdim=True))
                h = bs[c].index_copy(0, F["idx"], bs[c][F["idx"]] - Mn[:, c])
                newH.append(h.reshape(H[c].shape))
                newM.append(Mn)
            return newH, newM

        def e_step(E, H, n):
            curl = self._curl_h(H)
            J = [torch.zeros_like(E[c]) for c in range(3)]
            for comp, box, tab in self.sources:
                if n < len(tab):
                    i0, j0, k0_, ni, nj, nk = box
                    J[comp][k0_:k0_ + nk, j0:j0 + nj, i0:i0 + ni] += float(tab[n])
            return [coefs[c][0] * E[c] + coefs[c][1] * (curl[c] - J[c]) for c in range(3)]

        dV = self.d[0] * self.d[1] * self.d[2]
        fc = None if film_cells is None else torch.tensor(np.asarray(film_cells, dtype=bool))

        def film_energy(E, H):
            Ex, Ey, Ez = E
            Hx, Hy, Hz = H
            # per cell: mean over the four edges of E_c^2, over the two faces of H_c^2
            ex = (Ex[:-1, :-1, :] ** 2 + Ex[:-1, 1:, :] ** 2 + Ex[1:, :-1, :] ** 2 + Ex[1:, 1:, :] ** 2) / 4
            ey = (Ey[:-1, :, :-1] ** 2 + Ey[:-1, :, 1:] ** 2 + Ey[1:, :, :-1] ** 2 + Ey[1:, :, 1:] ** 2) / 4
            ez = (Ez[:, :-1, :-1] ** 2 + Ez[:, :-1, 1:] ** 2 + Ez[:, 1:, :-1] ** 2 + Ez[:, 1:, 1:] ** 2) / 4
            hx = (Hx[:, :, :-1] ** 2 + Hx[:, :, 1:] ** 2) / 2
            hy = (Hy[:, :-1, :] ** 2 + Hy[:, 1:, :] ** 2) / 2
            hz = (Hz[:-1, :, :] ** 2 + Hz[1:, :, :] ** 2) / 2
            dens = 0.5 * EPS0 * eps_cell * (ex + ey + ez) + 0.5 * MU0 * (hx + hy + hz)
            return (dens * fc).sum() * dV

        L = torch.zeros((), dtype=F64)
        for n in range(nsteps):
            H, M = half(E, H, M)
            E = e_step(E, H, n)
            H, M = half(E, H, M)
            if loss == "film_energy":
                if n + 1 > loss_from:
                    L = L + self.dt * film_energy(E, H)
            else:
                i, j, k = ijk
                L = L + float(weights[n]) * E[field][k, j, i]
        return L

    def gradients(self, nsteps, **kw):
        """The loss (float) and its gradients: dH0 (3,), deps over eps_box and
        dMs over ms_box ([k, j, i] numpy arrays)."""
        L = self.run(nsteps, **kw)
        params = [self.H0, self.eps_patch, self.ms_patch]
        g = torch.autograd.grad(L, params, allow_unused=True)
        out = [np.zeros(tuple(p.shape)) if gi is None else gi.detach().numpy() for p, gi in zip(params, g)]
        return {"loss": float(L.detach()), "dH0": out[0], "deps": out[1], "dMs": out[2]}
