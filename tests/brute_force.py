"""A second, deliberately naive transcription of one coupled time step, for
tiny lattices (8 x 8): plain Python loops over nodes and links, one block per
equation of the paper, every reading of the design notes written out where it
is used.  Test infrastructure: it is compared with the C oracle node by node
(tests/test_oracle_brute_force.py) and shares no code with it or with the GPU
library; both only read the same seeded problem description.

State layout: Python lists indexed [y][x]; populations f[s][a][y][x] (two flow
components, D2Q9 directions a = 0..8) and g[k][a][y][x] (species k, D2Q5
directions 0..4), stored as they arrive at a node after streaming.

Order of one step (Sec. 4.7, Steps 1-5, pull form of the previous streaming):
moments (Eq. 9, 23) -> liquid marks and shares in transit (Sec. 4.5) ->
effective masses (Eq. 12-13, 15) -> forces (Eq. 11, 14, 16 and a body force)
-> velocities (Eq. 17-19) -> homogeneous sources (Eq. 5, 27, 28) -> flow and
solute collisions (Eq. 6, 8, 20-22) -> heterogeneous link fluxes (Eq. 29-31,
A2) -> volume of pixel (Eq. 32-35) -> amendments (Sec. 4.5) -> streaming with
halfway bounce-back, reactive flux and the free outlet (Sec. 5.1).
"""
import math

# D2Q9 lattice vectors (Eq. 7); D2Q5 uses the first five
E = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
W9 = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4          # equilibrium weights (after Eq. 8)
WPP = [0.0] + [1 / 3] * 4 + [1 / 12] * 4            # pseudopotential weights (after Eq. 11)
FLUID, INERT, SOLID_D, SOLID_F = 0, 1, 2, 3
# solute held by a node at the start of a step
NONE, STREAM, HOLD, SHARE = 0, 1, 2, 3


def opposite(a):
    ex, ey = E[a]
    return E.index((-ex, -ey))


def _zeros(ny, nx, v=0.0):
    return [[v] * nx for _ in range(ny)]


class BruteForce:
    def __init__(self, prob):
        self.p = prob
        nx, ny = prob.nx, prob.ny
        self.nx, self.ny = nx, ny
        self.ns = prob.n_species
        self.type = [[int(prob.type0[y, x]) for x in range(nx)] for y in range(ny)]
        if prob.V0 is None:
            self.V = [[1.0 if self.type[y][x] in (SOLID_D, SOLID_F) else 0.0 for x in range(nx)] for y in range(ny)]
        else:
            self.V = [[float(prob.V0[y, x]) for x in range(nx)] for y in range(ny)]
        # initial liquid set: rho_1 above half the largest rho_1 (Sec. 4.5)
        rmax = max(float(prob.rho1[y, x]) for y in range(ny) for x in range(nx) if self.type[y][x] == FLUID)
        self.rho_max_prev = rmax
        self.f = [[_zeros(ny, nx) for _ in range(9)] for _ in range(2)]
        self.g = [[_zeros(ny, nx) for _ in range(5)] for _ in range(self.ns)]
        self.sflag = _zeros(ny, nx, NONE)
        self.stranded = _zeros(ny, nx, False)
        for y in range(ny):
            for x in range(nx):
                if self.type[y][x] != FLUID:
                    continue
                for a in range(9):      # rest equilibrium, Eq. 8 with u = 0
                    self.f[0][a][y][x] = W9[a] * float(prob.rho1[y, x])
                    self.f[1][a][y][x] = W9[a] * float(prob.rho2[y, x])
                if float(prob.rho1[y, x]) > prob.liquid_frac * rmax:
                    self.sflag[y][x] = STREAM
                    for k in range(self.ns):
                        for a in range(5):
                            self.g[k][a][y][x] = self.J(k, a) * float(prob.C0[k, y, x])
        self.ledger = dict(mass_src=[0.0, 0.0], mass_inj=[0.0, 0.0], mass_rem=[0.0, 0.0],
                           sol_src=[0.0] * self.ns, sol_het=[0.0] * self.ns, sol_rem=[0.0] * self.ns,
                           vol_dv=0.0, vol_clip=0.0, n_psi_clamp=0.0, n_dissolved=0.0,
                           n_precipitated=0.0, n_liq_to_gas=0.0, n_gas_to_liq=0.0, steps=0.0)

    # ------------------------------------------------------------ lattice
    def J(self, k, a):
        """Eq. 22: J_0 for the rest direction, (1 - J_0)/4 for the others."""
        J0 = self.p.species[k].J0
        return J0 if a == 0 else (1.0 - J0) / 4.0

    def neighbour(self, x, y, a, amendment=False):
        """The node at (x, y) + e_a: wrapped on a periodic side, None beyond a
        wall; beyond the free outlet on top a ghost row repeating the top row
        (Sec. 5.1), except for the amendments, which see no node there."""
        X, Y = x + E[a][0], y + E[a][1]
        if not 0 <= X < self.nx:
            if not self.p.periodic_x:
                return None
            X %= self.nx
        if Y >= self.ny and self.p.outlet_top:
            return None if amendment else (X, self.ny - 1)
        if not 0 <= Y < self.ny:
            if not self.p.periodic_y:
                return None
            Y %= self.ny
        return (X, Y)

    def through_outlet(self, y, a):
        return self.p.outlet_top and y + E[a][1] >= self.ny

    def fluid(self, node):
        return node is not None and self.type[node[1]][node[0]] == FLUID

    # ------------------------------------------------------------ physics
    def carnahan_starling(self, rho):
        """Eq. 12."""
        p = self.p
        e = p.b * rho / 4.0
        return rho * p.R * p.T * (1.0 + e + e * e - e ** 3) / (1.0 - e) ** 3 - p.a * rho * rho

    def step(self, n=1):
        for _ in range(n):
            self._step()

    def _step(self):
        p, nx, ny, ns = self.p, self.nx, self.ny, self.ns
        nodes = [(x, y) for y in range(ny) for x in range(nx)]
        led = self.ledger

        # Eq. 9 and 23: moments of the streamed populations
        rho = [_zeros(ny, nx), _zeros(ny, nx)]
        jx = [_zeros(ny, nx), _zeros(ny, nx)]
        jy = [_zeros(ny, nx), _zeros(ny, nx)]
        C = [_zeros(ny, nx) for _ in range(ns)]
        for (x, y) in nodes:
            if self.type[y][x] == FLUID or self.stranded[y][x]:
                for s in range(2):
                    for a in range(9):
                        v = self.f[s][a][y][x]
                        rho[s][y][x] += v
                        jx[s][y][x] += v * E[a][0]
                        jy[s][y][x] += v * E[a][1]
            if self.sflag[y][x] != NONE:
                for k in range(ns):
                    C[k][y][x] = sum(self.g[k][a][y][x] for a in range(5))

        # Sec. 4.5: liquid marks of this step against the previous maximum
        thr = p.liquid_frac * self.rho_max_prev
        liq = _zeros(ny, nx, False)
        for (x, y) in nodes:
            liq[y][x] = self.type[y][x] == FLUID and rho[0][y][x] > thr
        # shares in transit reach the nodes that were liquid when they were sent
        Cin = [_zeros(ny, nx) for _ in range(ns)]
        for (x, y) in nodes:
            if self.sflag[y][x] != STREAM:
                continue
            for a in range(1, 5):
                q = self.neighbour(x, y, a, amendment=True)
                if q is not None and self.sflag[q[1]][q[0]] == SHARE:
                    for k in range(ns):
                        Cin[k][y][x] += C[k][q[1]][q[0]]
        rmax_now = 0.0
        for (x, y) in nodes:
            if self.type[y][x] == FLUID:
                rmax_now = max(rmax_now, rho[0][y][x])
            if liq[y][x] and self.sflag[y][x] in (NONE, SHARE):
                for k in range(ns):          # newly liquid without content
                    C[k][y][x] = 0.0
                    for a in range(5):
                        self.g[k][a][y][x] = 0.0
            if self.sflag[y][x] == STREAM and not liq[y][x] and self.type[y][x] == FLUID:
                led["n_liq_to_gas"] += 1.0
            if liq[y][x] and self.sflag[y][x] != STREAM:
                led["n_gas_to_liq"] += 1.0

        # Eq. 12-13 (with the prefactor that matches the weights of Eq. 11) and Eq. 15
        psi, phi1, phi2 = _zeros(ny, nx), _zeros(ny, nx), _zeros(ny, nx)
        pre = p.psi_prefactor if p.psi_prefactor > 0 else 2.0
        for (x, y) in nodes:
            if self.type[y][x] != FLUID:
                continue
            r1, r2 = rho[0][y][x], rho[1][y][x]
            if p.G11 != 0.0:
                arg = pre * (self.carnahan_starling(r1) - r1 / 3.0) / p.G11
                if arg < 0.0:
                    arg = 0.0
                    led["n_psi_clamp"] += 1.0
                psi[y][x] = math.sqrt(arg)
            if p.rho20 > 0.0:
                phi1[y][x] = 1.0 - math.exp(-r2 / p.rho20)
            if p.rho10 > 0.0:
                phi2[y][x] = p.a0 - math.exp(-r1 / p.rho10)

        # Eq. 11 (cohesion), Eq. 14 (pair force), Eq. 16 (adhesion) and body force.
        # A neighbour that is not fluid counts s = 1 in Eq. 16 and lends the
        # potentials of its mirror image in the wall to Eq. 11 and 14: the centre
        # for an axis link; for a diagonal link the fluid axis neighbours that
        # share its column or its row (their mean if both are fluid), else the centre.
        Fx, Fy = [_zeros(ny, nx), _zeros(ny, nx)], [_zeros(ny, nx), _zeros(ny, nx)]
        for (x, y) in nodes:
            if self.type[y][x] != FLUID:
                continue
            sums = dict(psi=[0.0, 0.0], phi1=[0.0, 0.0], phi2=[0.0, 0.0], wall=[0.0, 0.0])
            for a in range(1, 9):
                q = self.neighbour(x, y, a)
                if self.fluid(q):
                    vals = (psi[q[1]][q[0]], phi1[q[1]][q[0]], phi2[q[1]][q[0]])
                    wall = 0.0
                else:
                    wall = 1.0
                    mirrors = [(x, y)]
                    if a >= 5:
                        qx = self.neighbour(x, y, 1 if E[a][0] > 0 else 3)
                        qy = self.neighbour(x, y, 2 if E[a][1] > 0 else 4)
                        fl = [m for m in (qx, qy) if self.fluid(m)]
                        if fl:
                            mirrors = fl
                    vals = tuple(sum(field[m[1]][m[0]] for m in mirrors) / len(mirrors)
                                 for field in (psi, phi1, phi2))
                for d in range(2):
                    sums["psi"][d] += WPP[a] * vals[0] * E[a][d]
                    sums["phi1"][d] += WPP[a] * vals[1] * E[a][d]
                    sums["phi2"][d] += WPP[a] * vals[2] * E[a][d]
                    sums["wall"][d] += WPP[a] * wall * E[a][d]
            r1, r2 = rho[0][y][x], rho[1][y][x]
            F = []
            for d in range(2):
                F1 = (-p.G11 * psi[y][x] * sums["psi"][d] - p.G12 * phi1[y][x] * sums["phi2"][d]
                      - p.w_adh[0] * psi[y][x] * sums["wall"][d] + r1 * p.gbody[d])
                F2 = -p.G21 * phi2[y][x] * sums["phi1"][d] - p.w_adh[1] * r2 * sums["wall"][d] + r2 * p.gbody[d]
                F.append((F1, F2))
            for s in range(2):
                Fx[s][y][x], Fy[s][y][x] = F[0][s], F[1][s]

        # Eq. 17-19: common velocity weighted by 1/tau, shifted equilibrium
        # velocities, physical velocity
        ueq = [[_zeros(ny, nx), _zeros(ny, nx)] for _ in range(2)]   # [s][d]
        ur = [_zeros(ny, nx), _zeros(ny, nx)]
        for (x, y) in nodes:
            if self.type[y][x] != FLUID:
                continue
            t1, t2 = p.tau
            r1, r2 = rho[0][y][x], rho[1][y][x]
            den = r1 / t1 + r2 / t2
            up = [(jx[0][y][x] / t1 + jx[1][y][x] / t2) / den, (jy[0][y][x] / t1 + jy[1][y][x] / t2) / den]
            for s in range(2):
                r = rho[s][y][x]
                Fs = (Fx[s][y][x], Fy[s][y][x])
                for d in range(2):
                    ueq[s][d][y][x] = up[d] + p.tau[s] * Fs[d] / r if r > 1e-12 else up[d]
            rt = r1 + r2
            ur[0][y][x] = (jx[0][y][x] + jx[1][y][x] + 0.5 * (Fx[0][y][x] + Fx[1][y][x])) / rt
            ur[1][y][x] = (jy[0][y][x] + jy[1][y][x] + 0.5 * (Fy[0][y][x] + Fy[1][y][x])) / rt

        # Eq. 5a, 5c (and first order), Eq. 27-28: sources at liquid nodes
        Ss = [_zeros(ny, nx), _zeros(ny, nx)]
        Sk = [_zeros(ny, nx) for _ in range(ns)]
        kinds = {"first_order", "r1_gas", "bimolecular"}
        for (x, y) in nodes:
            if not liq[y][x]:
                continue
            around = set()
            for a in range(1, 5):
                q = self.neighbour(x, y, a)
                if q is not None:
                    around.add(self.type[q[1]][q[0]])
            for r in p.hom:
                assert r.kind in kinds
                k_rate = r.k * r.surface_factor if any(t in around for t in r.surface) else r.k
                c = lambda i: C[i][y][x]  # noqa: E731
                if r.kind == "first_order":
                    R = k_rate * c(r.re[0])
                elif r.kind == "bimolecular":
                    R = k_rate * c(r.re[0]) * c(r.re[1])
                else:
                    gas = max(rho[1][y][x] / r.M_gas, 0.0)
                    R = k_rate * (c(r.re[0]) - c(r.pr[0]) * math.sqrt(gas) / r.K_eq)
                    Ss[0][y][x] -= 0.5 * R * r.M_gas
                    Ss[1][y][x] += 0.5 * R * r.M_gas
                for i in r.re:
                    if i >= 0:
                        Sk[i][y][x] -= R
                for i in r.pr:
                    if i >= 0:
                        Sk[i][y][x] += R
            for s in range(2):
                led["mass_src"][s] += Ss[s][y][x]
            for k in range(ns):
                led["sol_src"][k] += Sk[k][y][x]

        # Eq. 6 and 8: flow collision at fluid nodes
        fs = [[_zeros(ny, nx) for _ in range(9)] for _ in range(2)]
        for (x, y) in nodes:
            if self.type[y][x] != FLUID:
                continue
            for s in range(2):
                om = 1.0 / p.tau[s]
                ux, uy = ueq[s][0][y][x], ueq[s][1][y][x]
                for a in range(9):
                    eu = E[a][0] * ux + E[a][1] * uy
                    feq = W9[a] * rho[s][y][x] * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * (ux * ux + uy * uy))
                    fv = self.f[s][a][y][x]
                    fs[s][a][y][x] = fv - om * (fv - feq) + W9[a] * Ss[s][y][x]

        # Eq. 20-22: solute collision at liquid nodes with the physical velocity
        gs = [[_zeros(ny, nx) for _ in range(5)] for _ in range(ns)]
        for (x, y) in nodes:
            if not liq[y][x]:
                continue
            for k in range(ns):
                om = 1.0 / p.species[k].tau_g
                for a in range(5):
                    geq = C[k][y][x] * (self.J(k, a) + 0.5 * (E[a][0] * ur[0][y][x] + E[a][1] * ur[1][y][x]))
                    gv = self.g[k][a][y][x]
                    gs[k][a][y][x] = gv - om * (gv - geq) + self.J(k, a) * Sk[k][y][x]

        # Eq. 29-31, A2: link flux of each surface reaction at a liquid node,
        # halfway-wall Robin form with D of Eq. 24
        Phi = [_zeros(ny, nx) for _ in p.het]
        for ri, r in enumerate(p.het):
            sp = p.species[r.reactant]
            D = 0.5 * (1.0 - sp.J0) * (sp.tau_g - 0.5)
            kap = 2.0 * D * r.k / (2.0 * D + r.k) if 2.0 * D + r.k > 0 else 0.0
            for (x, y) in nodes:
                if liq[y][x]:
                    v = kap * (C[r.reactant][y][x] - r.C_eq)
                    Phi[ri][y][x] = max(v, 0.0) if r.irreversible else v

        # Eq. 32-35: volume of pixel
        tnext = [row[:] for row in self.type]
        for (x, y) in nodes:
            t = self.type[y][x]
            if t in (SOLID_D, SOLID_F):
                dv, touched = 0.0, False
                for a in range(1, 5):
                    q = self.neighbour(x, y, a)
                    if not (self.fluid(q) and liq[q[1]][q[0]]):
                        continue
                    for ri, r in enumerate(p.het):
                        if t not in r.surface:
                            continue
                        if r.mode == "consumes":
                            dv -= r.molar_volume * Phi[ri][q[1]][q[0]]
                            touched = True
                        elif r.mode == "mineral":
                            dv += r.molar_volume * Phi[ri][q[1]][q[0]]
                            touched = True
                if touched:
                    self.V[y][x] += dv
                    led["vol_dv"] += dv
                if self.V[y][x] <= 0.0:
                    if any(self.fluid(self.neighbour(x, y, a, amendment=True)) for a in range(1, 9)):
                        tnext[y][x] = FLUID
            elif t == FLUID and liq[y][x]:
                dv, touched = 0.0, False
                for a in range(1, 5):
                    q = self.neighbour(x, y, a)
                    if q is None or self.type[q[1]][q[0]] not in (SOLID_D, SOLID_F):
                        continue
                    for ri, r in enumerate(p.het):
                        if self.type[q[1]][q[0]] in r.surface and r.mode == "grows":
                            dv += r.molar_volume * Phi[ri][y][x]
                            touched = True
                if touched:
                    self.V[y][x] += dv
                    led["vol_dv"] += dv
                if self.V[y][x] >= 1.0:
                    tnext[y][x] = SOLID_F

        # Sec. 4.5 amendments
        def fluid_count(x, y):
            return sum(1 for b in range(1, 9) if self.fluid(self.neighbour(x, y, b, amendment=True)))

        for (x, y) in nodes:
            # (a) stranded populations go, at rest, to the fluid D2Q9 neighbours
            if self.type[y][x] == FLUID:
                give = [0.0, 0.0]
                for a in range(1, 9):
                    q = self.neighbour(x, y, a, amendment=True)
                    if q is None or not self.stranded[q[1]][q[0]]:
                        continue
                    m = fluid_count(*q)
                    for s in range(2):
                        give[s] += rho[s][q[1]][q[0]] / m
                for s in range(2):
                    if give[s] != 0.0:
                        for a in range(9):
                            fs[s][a][y][x] += W9[a] * give[s]
            # (b) shares taken by receivers that are liquid now, at rest
            if liq[y][x] and self.sflag[y][x] == STREAM:
                for k in range(ns):
                    if Cin[k][y][x] != 0.0:
                        for a in range(5):
                            gs[k][a][y][x] += self.J(k, a) * Cin[k][y][x]
        snext = _zeros(ny, nx, NONE)
        sent = {}
        for (x, y) in nodes:
            if self.stranded[y][x] and fluid_count(x, y) == 0:
                for s in range(2):
                    led["mass_rem"][s] += rho[s][y][x]
            # (b) a node holding solute that is not liquid now splits its content
            # (with what it received) among its liquid D2Q5 neighbours, or keeps it
            snext[y][x] = STREAM if liq[y][x] else NONE
            if not liq[y][x] and self.sflag[y][x] in (STREAM, HOLD) and ns > 0:
                m = sum(1 for b in range(1, 5)
                        if (lambda q: q is not None and liq[q[1]][q[0]])(self.neighbour(x, y, b, amendment=True)))
                content = []
                for k in range(ns):
                    c = C[k][y][x] + (Cin[k][y][x] if self.sflag[y][x] == STREAM else 0.0)
                    content.append(c / m if m > 0 else c)
                sent[(x, y)] = content
                if any(c != 0.0 for c in content):
                    snext[y][x] = SHARE if m > 0 else HOLD
        # (c) nodes freed by dissolution start at rest with the mean density of
        # their fluid D2Q9 neighbours
        rbar = {}
        for (x, y) in nodes:
            if self.type[y][x] != FLUID and tnext[y][x] == FLUID:
                nbrs = [q for q in (self.neighbour(x, y, a, amendment=True) for a in range(1, 9)) if self.fluid(q)]
                rb = [sum(rho[s][q[1]][q[0]] for q in nbrs) / len(nbrs) for s in range(2)]
                rbar[(x, y)] = rb
                for s in range(2):
                    led["mass_inj"][s] += rb[s]
                led["n_dissolved"] += 1.0
                led["vol_clip"] += self.V[y][x]

        # streaming (Eq. 6, 20 left-hand sides) with halfway bounce-back
        fn = [[_zeros(ny, nx) for _ in range(9)] for _ in range(2)]
        gn = [[_zeros(ny, nx) for _ in range(5)] for _ in range(ns)]
        for (x, y) in nodes:
            if self.type[y][x] != FLUID:
                continue
            for a in range(9):
                q = self.neighbour(x, y, a)
                for s in range(2):
                    if self.fluid(q):
                        if not self.through_outlet(y, a):
                            fn[s][a][q[1]][q[0]] = fs[s][a][y][x]
                    else:
                        fn[s][opposite(a)][y][x] = fs[s][a][y][x]
        if p.outlet_top:
            y = ny - 1
            for x in range(nx):
                if self.type[y][x] != FLUID:
                    continue
                for a in range(1, 9):
                    if E[a][1] >= 0:
                        continue
                    q = self.neighbour(x, y, opposite(a))   # the ghost sender's model node
                    if self.fluid(q):
                        for s in range(2):
                            fn[s][a][y][x] = fs[s][a][q[1]][q[0]]
        for (x, y) in nodes:
            if not liq[y][x]:
                continue
            for k in range(ns):
                for a in range(5):
                    q = self.neighbour(x, y, a)
                    v = gs[k][a][y][x]
                    if q is not None and liq[q[1]][q[0]]:
                        if not self.through_outlet(y, a):
                            gn[k][a][q[1]][q[0]] = v
                        continue
                    if q is not None and self.type[q[1]][q[0]] in (SOLID_D, SOLID_F):
                        for ri, r in enumerate(p.het):
                            if self.type[q[1]][q[0]] not in r.surface:
                                continue
                            if r.reactant == k:
                                v -= Phi[ri][y][x]
                                led["sol_het"][k] -= Phi[ri][y][x]
                            if r.product == k:
                                v += Phi[ri][y][x]
                                led["sol_het"][k] += Phi[ri][y][x]
                    gn[k][opposite(a)][y][x] = v
        if p.outlet_top:
            y = ny - 1
            for x in range(nx):
                if liq[y][x]:
                    for k in range(ns):
                        gn[k][4][y][x] = gs[k][4][y][x]
        for (x, y), rb in rbar.items():
            for s in range(2):
                for a in range(9):
                    fn[s][a][y][x] = W9[a] * rb[s]
        for (x, y), content in sent.items():
            for k in range(ns):
                for a in range(5):
                    gn[k][a][y][x] = self.J(k, a) * content[k]

        # the next state
        for (x, y) in nodes:
            told, tnew = self.type[y][x], tnext[y][x]
            if told == FLUID and tnew == SOLID_F:
                led["n_precipitated"] += 1.0
            if told != FLUID and tnew == FLUID:
                self.V[y][x] = 0.0
            self.stranded[y][x] = told == FLUID and tnew == SOLID_F
            self.type[y][x] = tnew
        self.sflag = snext
        self.f, self.g = fn, gn
        self.rho_max_prev = rmax_now
        led["steps"] += 1.0
        self.liq = liq

    # ------------------------------------------------------------ read-out
    def densities_and_content(self):
        """rho_1, rho_2 (Eq. 9), this step's liquid marks and the solute each
        node holds once the shares in transit are delivered (Sec. 4.5), for
        comparison with the oracle's field export."""
        p, nx, ny, ns = self.p, self.nx, self.ny, self.ns
        rho = [_zeros(ny, nx), _zeros(ny, nx)]
        C = [_zeros(ny, nx) for _ in range(ns)]
        for y in range(ny):
            for x in range(nx):
                if self.type[y][x] == FLUID or self.stranded[y][x]:
                    for s in range(2):
                        rho[s][y][x] = sum(self.f[s][a][y][x] for a in range(9))
                if self.sflag[y][x] != NONE:
                    for k in range(ns):
                        C[k][y][x] = sum(self.g[k][a][y][x] for a in range(5))
        thr = p.liquid_frac * self.rho_max_prev
        liq = [[self.type[y][x] == FLUID and rho[0][y][x] > thr for x in range(nx)] for y in range(ny)]
        out = [_zeros(ny, nx) for _ in range(ns)]
        for y in range(ny):
            for x in range(nx):
                sf = self.sflag[y][x]
                for k in range(ns):
                    if sf == HOLD:
                        out[k][y][x] = C[k][y][x]
                    elif sf == STREAM:
                        c = C[k][y][x]
                        for a in range(1, 5):
                            q = self.neighbour(x, y, a, amendment=True)
                            if q is not None and self.sflag[q[1]][q[0]] == SHARE:
                                c += C[k][q[1]][q[0]]
                        out[k][y][x] = c
        return rho, liq, out
