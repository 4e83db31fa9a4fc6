"""Pure-Python brute-force stepper for tiny PEC boxes (test infrastructure).

An independent second implementation of the coupled Yee + LLG step of
arXiv:2510.22221 (Methods, "Numerical Model"), used only to pin the C oracle
on grids of a few cells.  It shares nothing with the C oracle: every Yee
site is addressed by its *doubled* coordinate (X, Y, Z) = 2 x position / d,
so cell centres are odd-odd-odd, E_c sites have exactly one odd coordinate
(the c axis) and H_c sites exactly two (all but the c axis).  Neighbours are
then +-1 in doubled coordinates and every rule below is written in that
form, directly from the equations:

  * H/M half step (eq. iterate_H with the trapezoidal LLG, eqs.
    llg_tra4-llg_tra6, normalised to Ms), then the E step (the semi-implicit
    Ampere update), then the second H/M half step;
  * the field at a magnetic face is B^ = H + M; the two transverse B^
    components come from the mean of the nearest sites of those families;
  * PEC walls on every face; no PML, no periodic axes.
"""
from __future__ import annotations

import math

MU0 = 4e-7 * math.pi
C0 = 299792458.0
EPS0 = 1.0 / (MU0 * C0 * C0)


def _odd(v):
    return v % 2 == 1


class Brute:
    def __init__(self, n, d, dt, table, ids, H0, mdir):
        """n = (nx, ny, nz); ids[k][j][i] material index; table rows are
        (eps_r, sigma, is_pec, Ms, alpha, |gamma|)."""
        self.n = tuple(n)
        self.d = tuple(d)
        self.dt = dt
        self.table = table
        self.H0 = tuple(H0)
        self.lim = tuple(2 * v for v in n)
        self.cell = {}
        for k in range(n[2]):
            for j in range(n[1]):
                for i in range(n[0]):
                    self.cell[(2 * i + 1, 2 * j + 1, 2 * k + 1)] = int(ids[k][j][i])
        self.E, self.H = {}, {}
        for X in range(self.lim[0] + 1):
            for Y in range(self.lim[1] + 1):
                for Z in range(self.lim[2] + 1):
                    nodd = _odd(X) + _odd(Y) + _odd(Z)
                    if nodd == 1:
                        self.E[(X, Y, Z)] = 0.0
                    elif nodd == 2:
                        self.H[(X, Y, Z)] = 0.0
        self.M = {}
        self.ms = {}
        self.al = {}
        self.ga = {}
        for s in self.H:
            c = self.comp_h(s)
            cells = [m for m in (self.cell.get(self.shift(s, c, -1)), self.cell.get(self.shift(s, c, +1)))
                     if m is not None]
            ms = sum(table[m][3] for m in cells) / len(cells)
            mag = [m for m in cells if table[m][3] > 0]
            if ms > 0:
                self.ms[s] = ms
                self.al[s] = sum(table[m][4] for m in mag) / len(mag)
                self.ga[s] = sum(table[m][5] for m in mag) / len(mag)
                nu = math.sqrt(sum(u * u for u in mdir))
                self.M[s] = [ms * u / nu for u in mdir]
        self.M0 = {s: list(v) for s, v in self.M.items()}
        self.coef = {}
        for s in self.E:
            c = self.comp_e(s)
            wall = any(s[a] in (0, self.lim[a]) for a in range(3) if a != c)
            a1, a2 = [a for a in range(3) if a != c]
            cells = []
            for u in (-1, 1):
                for v in (-1, 1):
                    q = list(s)
                    q[a1] += u
                    q[a2] += v
                    m = self.cell.get(tuple(q))
                    if m is not None:
                        cells.append(m)
            pec = wall or any(table[m][2] for m in cells)
            if pec:
                self.coef[s] = None
                continue
            eps = EPS0 * sum(table[m][0] for m in cells) / len(cells)
            sig = sum(table[m][1] for m in cells) / len(cells)
            self.coef[s] = ((eps / dt - sig / 2) / (eps / dt + sig / 2), 1.0 / (eps / dt + sig / 2))
        self.sources = []
        self.step_n = 0

    # --- site helpers -----------------------------------------------------
    @staticmethod
    def comp_e(s):
        return [a for a in range(3) if _odd(s[a])][0]

    @staticmethod
    def comp_h(s):
        return [a for a in range(3) if not _odd(s[a])][0]

    @staticmethod
    def shift(s, a, v):
        q = list(s)
        q[a] += v
        return tuple(q)

    def add_source(self, comp, sites, table):
        """sites: list of doubled coordinates of E_comp edges."""
        self.sources.append((comp, set(sites), list(table)))

    # --- curls -------------------------------------------------------------
    def curl_e(self, s):
        c = self.comp_h(s)
        a1, a2 = (c + 1) % 3, (c + 2) % 3
        # d_{a1} E_{a2} - d_{a2} E_{a1}
        t1 = (self.E.get(self.shift(s, a1, +1), 0.0) - self.E.get(self.shift(s, a1, -1), 0.0)) / self.d[a1]
        t2 = (self.E.get(self.shift(s, a2, +1), 0.0) - self.E.get(self.shift(s, a2, -1), 0.0)) / self.d[a2]
        return t1 - t2

    def curl_h(self, s):
        c = self.comp_e(s)
        a1, a2 = (c + 1) % 3, (c + 2) % 3
        t1 = (self.H.get(self.shift(s, a1, +1), 0.0) - self.H.get(self.shift(s, a1, -1), 0.0)) / self.d[a1]
        t2 = (self.H.get(self.shift(s, a2, +1), 0.0) - self.H.get(self.shift(s, a2, -1), 0.0)) / self.d[a2]
        return t1 - t2

    # --- one H/M half step ------------------------------------------------------
    def half(self):
        k0 = MU0 * self.dt / 4.0
        bn, bs = {}, {}
        for s in self.H:
            c = self.comp_h(s)
            b = self.H[s] + (self.M[s][c] if s in self.M else 0.0)
            bn[s] = b
            bs[s] = b - self.dt / (2 * MU0) * self.curl_e(s)
        newH, newM = {}, {}
        for s in self.H:
            if s not in self.M:
                newH[s] = bs[s]
                continue
            c = self.comp_h(s)
            P = [0.0, 0.0, 0.0]
            Q = [0.0, 0.0, 0.0]
            P[c], Q[c] = bs[s], bn[s]
            for cp in range(3):
                if cp == c:
                    continue
                near = []
                for u in (-1, 1):
                    for v in (-1, 1):
                        q = self.shift(self.shift(s, c, u), cp, v)
                        if q in self.H:
                            near.append(q)
                P[cp] = sum(bs[q] for q in near) / len(near)
                Q[cp] = sum(bn[q] for q in near) / len(near)
            P = [P[w] + self.H0[w] for w in range(3)]
            Q = [Q[w] + self.H0[w] for w in range(3)]
            M = self.M[s]
            kk = k0 * self.ga[s]
            al, ms = self.al[s], self.ms[s]
            MxQ = [M[1] * Q[2] - M[2] * Q[1], M[2] * Q[0] - M[0] * Q[2], M[0] * Q[1] - M[1] * Q[0]]
            b = [M[w] - kk * MxQ[w] for w in range(3)]
            a = [-(kk * P[w] + al / ms * M[w]) for w in range(3)]
            ab = sum(a[w] * b[w] for w in range(3))
            aa = sum(a[w] * a[w] for w in range(3))
            axb = [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]
            X = [(b[w] + ab * a[w] - axb[w]) / (1 + aa) for w in range(3)]
            nx = math.sqrt(sum(v * v for v in X))
            Mn = [ms * v / nx for v in X]
            newM[s] = Mn
            newH[s] = bs[s] - Mn[c]
        self.H = newH
        self.M.update(newM)

    def e_step(self):
        newE = {}
        for s in self.E:
            cf = self.coef[s]
            if cf is None:
                newE[s] = self.E[s]
                continue
            c = self.comp_e(s)
            J = 0.0
            for comp, sites, tab in self.sources:
                if comp == c and s in sites and self.step_n < len(tab):
                    J += tab[self.step_n]
            newE[s] = cf[0] * self.E[s] + cf[1] * (self.curl_h(s) - J)
        self.E = newE

    def step(self, nsteps):
        for _ in range(nsteps):
            self.half()
            self.e_step()
            self.half()
            self.step_n += 1

    # --- export in natural index order ------------------------------------------
    def field_e(self, c):
        """E_c as nested lists [k][j][i] over the natural Yee index ranges."""
        return self._export(self.E, c, lambda a: a == c)

    def field_h(self, c):
        return self._export(self.H, c, lambda a: a != c)

    def _export(self, store, c, half_axis):
        dims = [self.n[a] if half_axis(a) else self.n[a] + 1 for a in range(3)]
        out = []
        for k in range(dims[2]):
            plane = []
            for j in range(dims[1]):
                row = []
                for i in range(dims[0]):
                    idx = (i, j, k)
                    s = tuple(2 * idx[a] + (1 if half_axis(a) else 0) for a in range(3))
                    row.append(store[s])
                plane.append(row)
            out.append(plane)
        return out

    def field_dm(self, c):
        """M - M0 on the family-c faces, [w][k][j][i]."""
        dims = [self.n[a] + 1 if a == c else self.n[a] for a in range(3)]
        out = []
        for w in range(3):
            vol = []
            for k in range(dims[2]):
                plane = []
                for j in range(dims[1]):
                    row = []
                    for i in range(dims[0]):
                        idx = (i, j, k)
                        s = tuple(2 * idx[a] + (0 if a == c else 1) for a in range(3))
                        row.append(self.M[s][w] - self.M0[s][w] if s in self.M else 0.0)
                    plane.append(row)
                vol.append(plane)
            out.append(vol)
        return out
