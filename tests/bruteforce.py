"""Exact-rational MPDATA on tiny grids (Python Fractions, dictionaries).

An independent second coding of the step (donor-cell pass, pseudo-velocity
with cross and third-order terms, limiter, infinite gauge), written without
arrays or strides so that an indexing or boundary mistake in the C oracle
shows up as a disagreement.  Every operation on the path is +, -, *, /, min,
max or abs, so the result is exact; the oracle must agree to FP64 rounding.
"""
from fractions import Fraction
from itertools import product


class Grid:
    def __init__(self, shape, bc):
        self.shape = tuple(shape)
        self.nd = len(shape)
        self.bc = [bc] * self.nd if isinstance(bc, int) else list(bc)

    def cell(self, p):
        out = []
        for d, q in enumerate(p):
            n = self.shape[d]
            out.append(q % n if self.bc[d] == 0 else min(max(q, 0), n - 1))
        return tuple(out)

    def wall(self, d, p):
        out = []
        for t, q in enumerate(p):
            n = self.shape[t]
            if t == d:
                out.append(q % n if self.bc[t] == 0 else min(max(q, 0), n))
            else:
                out.append(q % n if self.bc[t] == 0 else min(max(q, 0), n - 1))
        return tuple(out)

    def cells(self):
        return product(*[range(n) for n in self.shape])

    def walls(self, d):
        return product(*[range(n + (1 if t == d else 0)) for t, n in enumerate(self.shape)])


def _add(p, d, s):
    q = list(p)
    q[d] += s
    return tuple(q)


def _fr(num, den, iga, m):
    if iga:
        return num / m
    return Fraction(0) if den == 0 else num / den


def mpdata_exact(psi, c, g, shape, bc, n_iters, fct, iga, tot, n_steps, absf=False, dfl=False):
    """psi: dict cell->Fraction; c: list of dict wall->Fraction; g: dict or None."""
    G = Grid(shape, bc)
    one = Fraction(1)

    def X(f, p):
        return f[G.cell(p)]

    def W(f, d, p):
        return f[d][G.wall(d, p)]

    def Gv(p):
        return one if g is None else g[G.cell(p)]

    def donor(x, vel, flux_is_vel):
        out = {}
        for p in G.cells():
            acc = Fraction(0)
            for d in range(G.nd):
                fl = []
                for s in (0, 1):
                    w = _add(p, d, s)
                    v = W(vel, d, w)
                    if flux_is_vel:
                        fl.append(v)
                    else:
                        fl.append(max(v, 0) * X(x, _add(w, d, -1)) + min(v, 0) * X(x, w))
                acc += fl[1] - fl[0]
            out[p] = X(x, p) - acc / Gv(p)
        return out

    def pseudo(x, cp):
        if absf:                  # |psi| in every psi-fraction
            x = {k: abs(v) for k, v in x.items()}
        V = []
        for d in range(G.nd):
            Vd = {}
            for w in G.walls(d):
                L, R = _add(w, d, -1), w
                u = W(cp, d, w)
                gb = (Gv(L) + Gv(R)) / 2
                xl, xr = X(x, L), X(x, R)
                v = (abs(u) - u * u / gb) * _fr(xr - xl, xr + xl, iga, 2)
                cb = {}
                for o in range(G.nd):
                    if o == d:
                        continue
                    cb[o] = (W(cp, o, L) + W(cp, o, _add(L, o, 1)) + W(cp, o, R)
                             + W(cp, o, _add(R, o, 1))) / 4
                    a, b = X(x, _add(R, o, 1)), X(x, _add(L, o, 1))
                    e, f = X(x, _add(R, o, -1)), X(x, _add(L, o, -1))
                    v -= u * cb[o] / (2 * gb) * _fr(a + b - e - f, a + b + e + f, iga, 4)
                if dfl:                # divergent-flow term
                    dv = Fraction(0)
                    for o in range(G.nd):
                        for S in (L, R):
                            dv += W(cp, o, _add(S, o, 1)) - W(cp, o, S)
                    if iga:            # unit-field flux: times the wall mean of psi
                        dv = dv * (xl + xr) / 2
                    v -= u / (2 * gb) * dv / 2
                if tot:
                    x2, x_1 = X(x, _add(R, d, 1)), X(x, _add(L, d, -1))
                    Dq = _fr(x2 - xr - xl + x_1, x2 + xr + xl + x_1, iga, 4)
                    v += (3 * u * abs(u) / gb - 2 * u ** 3 / gb ** 2 - u) / 3 * Dq
                    for o in cb:
                        a, b = X(x, _add(R, o, 1)), X(x, _add(L, o, 1))
                        e, f = X(x, _add(R, o, -1)), X(x, _add(L, o, -1))
                        Eq = _fr(a - b - e + f, a + b + e + f, iga, 4)
                        v += (abs(u) * cb[o] / gb - 2 * u * u * cb[o] / gb ** 2) * Eq
                    if G.nd == 3:
                        o1, o2 = [o for o in range(3) if o != d]
                        num = den = Fraction(0)
                        for S in (L, R):
                            vals = {}
                            for s1, s2 in product((1, -1), (1, -1)):
                                vals[(s1, s2)] = X(x, _add(_add(S, o1, s1), o2, s2))
                            num += vals[(1, 1)] - vals[(-1, 1)] - vals[(1, -1)] + vals[(-1, -1)]
                            den += sum(vals.values())
                        v += Fraction(-2, 3) * u * cb[o1] * cb[o2] / gb ** 2 * _fr(num, den, iga, 8)
                Vd[w] = v
            V.append(Vd)
        return V

    def limit(psin, x, V):
        bu, bd = {}, {}
        for p in G.cells():
            nb = [p] + [_add(p, d, s) for d in range(G.nd) for s in (-1, 1)]
            vals = [X(psin, q) for q in nb] + [X(x, q) for q in nb]
            mx, mn = max(vals), min(vals)
            fin = fout = Fraction(0)
            for d in range(G.nd):
                vlo, vhi = W(V, d, p), W(V, d, _add(p, d, 1))
                wm = one if iga else X(x, _add(p, d, -1))
                wp = one if iga else X(x, _add(p, d, 1))
                wi = one if iga else X(x, p)
                fin += max(vlo, 0) * wm - min(vhi, 0) * wp
                fout += max(vhi, 0) * wi - min(vlo, 0) * wi
            bu[p] = Gv(p) * (mx - X(x, p)) / fin if fin > 0 else one
            bd[p] = Gv(p) * (X(x, p) - mn) / fout if fout > 0 else one
        out = []
        for d in range(G.nd):
            Od = {}
            for w in G.walls(d):
                L, R = _add(w, d, -1), w
                v = W(V, d, w)
                Od[w] = (max(v, 0) * min(one, X(bd, L), X(bu, R))
                         + min(v, 0) * min(one, X(bu, L), X(bd, R)))
            out.append(Od)
        return out

    for _ in range(n_steps):
        psin = psi
        y = donor(psin, c, False)
        cp = c
        for _it in range(2, n_iters + 1):
            x = y
            V = pseudo(x, cp)
            if fct:
                V = limit(psin, x, V)
            y = donor(x, V, iga)
            cp = V
        psi = y
    return psi
