"""Reference (oracle) implementation of the full-order implicit cell step.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the HIP path and is never used to produce a product result.

What it computes (arXiv 1704.04139, MULTIBAT):
  * Sec. 2.2, eqs. (2.1)-(2.7): solid Li diffusion and charge conservation,
    electrolyte mass and charge conservation with migration and the
    concentration-gradient (dmu/dc) term, Butler-Volmer intercalation law with
    alpha = 1/2 and no (c_max - c)^alpha factor, interface conditions with the
    normal pointing from solid into electrolyte, Table "interface conditions".
  * Sec. 2.3, eqs. (2.8)-(2.12): plating/stripping Butler-Volmer law with the
    regularisation f_pre(n) = n^4/(n_c^4 + n^4), plating overpotential
    Phi_Pl - phi_El, interface current equal to the stripping current.
  * Sec. 2.4, eq. (2.13): cell-centred finite volumes on the uniform voxel
    grid, Butler-Volmer laws as the numerical flux on phase faces, implicit
    Euler in time, one concentration and one potential unknown per voxel.
  * Sec. 2.5 (output functionals): cell voltage and mean solid concentration.

Readings where the paper is silent: full cell with
the cathode following the same intercalation law; constant coefficients;
the 1/c term discretised as RT (ln c_k - ln c_i)/h with thermodynamic factor
theta; BV evaluated from the two adjacent cell values; per-face plated amount
n_f on every anode/pore face, plating in parallel with intercalation, plated
metal at the adjacent anode voxel's potential; collector planes at z = 0
(anode, phi = 0 over half a voxel) and z = L (cathode, uniform galvanostatic
flux over its solid faces); zero flux on the lateral sides.

Precision: float64 throughout.  Linear solves: SciPy SuperLU (splu) inside a
damped Newton iteration; single-threaded when the caller pins BLAS threads.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

FARADAY = 96485.33212      # C/mol (CODATA 2018)
GAS_R = 8.314462618        # J/(mol K) (CODATA 2018)

PORE, ANODE, CATHODE = 0, 1, 2
FOIL = 3            # Li-metal counter electrode of a half cell (Sec. 2.2), held in the cathode slot
# direction index seen from a voxel: 0:-x 1:+x 2:-y 3:+y 4:-z 5:+z
_AXIS_DIRS = ((0, 1), (2, 3), (4, 5))


class Geometry:
    """Face lists of a labelled voxel grid (Sec. 2.4: every face of the
    uniform grid carries one numerical flux)."""

    def __init__(self, labels: np.ndarray):
        lab = np.ascontiguousarray(labels, dtype=np.uint8)
        if lab.ndim != 3:
            raise ValueError("labels must be (nz, ny, nx)")
        self.nz, self.ny, self.nx = lab.shape
        self.N = lab.size
        flat = lab.ravel()
        if np.any(flat > FOIL):
            raise ValueError("labels must be 0 (pore), 1 (anode), 2 (cathode) or 3 (Li foil)")
        # a half cell (graphite against a Li foil, Sec. 2.2) holds its foil in
        # the counter-electrode slot; a cell is either full or half
        self.half = bool(np.any(flat == FOIL))
        if self.half and np.any(flat == CATHODE):
            raise ValueError("a cell holds either cathode (2) or Li foil (3) voxels, not both")
        self.lab = np.where(flat == FOIL, CATHODE, flat).astype(np.uint8)
        idx = np.arange(self.N).reshape(lab.shape)
        lo_list, hi_list, ax_list = [], [], []
        for axis, sl_lo, sl_hi in ((0, np.s_[:, :, :-1], np.s_[:, :, 1:]),
                                   (1, np.s_[:, :-1, :], np.s_[:, 1:, :]),
                                   (2, np.s_[:-1, :, :], np.s_[1:, :, :])):
            lo = idx[sl_lo].ravel()
            hi = idx[sl_hi].ravel()
            lo_list.append(lo)
            hi_list.append(hi)
            ax_list.append(np.full(lo.size, axis, dtype=np.int64))
        lo = np.concatenate(lo_list)
        hi = np.concatenate(hi_list)
        ax = np.concatenate(ax_list)
        la, lb = self.lab[lo], self.lab[hi]
        if np.any(((la == ANODE) & (lb == CATHODE)) | ((la == CATHODE) & (lb == ANODE))):
            raise ValueError("the two electrodes may not share a face (no such interface, Sec. 2.2)")
        pp = (la == PORE) & (lb == PORE)
        self.pp_lo, self.pp_hi = lo[pp], hi[pp]
        ss = (la != PORE) & (la == lb)
        self.ss_lo, self.ss_hi = lo[ss], hi[ss]
        self.ss_phase = la[ss].astype(np.int64)
        # interface faces: (solid voxel, pore voxel, direction seen from the solid)
        s_lo = (la != PORE) & (lb == PORE)
        s_hi = (la == PORE) & (lb != PORE)
        solid = np.concatenate([lo[s_lo], hi[s_hi]])
        pore = np.concatenate([hi[s_lo], lo[s_hi]])
        dirs = np.concatenate([np.array([_AXIS_DIRS[a][1] for a in ax[s_lo]], dtype=np.int64),
                               np.array([_AXIS_DIRS[a][0] for a in ax[s_hi]], dtype=np.int64)])
        order = np.lexsort((dirs, solid))       # canonical: by solid voxel, then direction
        self.if_s, self.if_p, self.if_dir = solid[order], pore[order], dirs[order]
        self.if_phase = self.lab[self.if_s].astype(np.int64)
        # plating faces = anode interface faces, in canonical order
        self.pl_face = np.nonzero(self.if_phase == ANODE)[0]
        self.F_if = self.if_s.size
        self.F_pl = self.pl_face.size
        k = idx // (self.nx * self.ny)
        kf = k.ravel()
        self.bot = np.nonzero((kf == 0) & (self.lab == ANODE))[0]
        self.top = np.nonzero((kf == self.nz - 1) & (self.lab == CATHODE))[0]
        if self.bot.size == 0 or self.top.size == 0:
            raise ValueError("each collector plane needs solid of its electrode")


def ocp(a: tuple, x):
    """Open-circuit potential U(x) = a0 + a1 ln((1-x)/x) (synthetic, monotone)."""
    return a[0] + a[1] * np.log((1.0 - x) / x)


def docp(a: tuple, x):
    """dU/dx."""
    return -a[1] / (x * (1.0 - x))


def f_pre(n, n_c):
    """Sec. 2.3 regularisation n^4/(n_c^4 + n^4)."""
    n4 = n ** 4
    return n4 / (n_c ** 4 + n4)


def df_pre(n, n_c):
    c4 = n_c ** 4
    return 4.0 * n ** 3 * c4 / (c4 + n ** 4) ** 2


class Model:
    """Discrete residual F(u; u_old) of eq. (2.13) and its analytic Jacobian.

    Unknown vector u = [c (N), phi (N), n (F_pl)]; residual rows
      R^c_i = V (c_i - c_i^old)/dt + A sum_f N_out   (mol/s)
      R^p_i = A sum_f j_out                           (A)
      R^n_f = A (n_f - n_f^old)/dt + A i_pl/F         (mol/s)
    """

    def __init__(self, geom: Geometry, prm: dict):
        self.g = geom
        self.p = dict(prm)
        p = self.p
        self.h = p["h"]
        self.A = self.h ** 2
        self.V = self.h ** 3
        self.RT = GAS_R * p["T"]
        self.beta = FARADAY / (2.0 * self.RT)
        # Li foil (half cell): no Li diffusion or intercalation in the metal
        self.half = geom.half
        self.Ds = {ANODE: p["Ds_an"], CATHODE: 0.0 if self.half else p["Ds_ca"]}
        self.sig = {ANODE: p["sigma_an"], CATHODE: p["sigma_ca"]}
        self.cmax = {ANODE: p["cmax_an"], CATHODE: p["cmax_ca"]}
        self.i00 = {ANODE: p["i00_an"], CATHODE: p["i00_ca"]}
        self.U = {ANODE: tuple(p["U_an"]), CATHODE: tuple(p["U_ca"])}
        g = geom
        self.mu = p["I_app"] / (g.nx * g.ny * self.A)          # applied current density
        self.mu_ref = max(abs(self.mu), 1.0)
        self.c_ref = np.where(g.lab == PORE, p["c0"],
                              np.where(g.lab == ANODE, p["cmax_an"], p["cmax_ca"])).astype(float)
        self.N = g.N
        self.n_unknowns = 2 * g.N + g.F_pl

    # ------------------------------------------------------------------ state
    def initial_state(self):
        """Zero-current equilibrium (reading of eq. (2.13)'s c^(0) = c_0 with
        the potentials that make every interface flux vanish)."""
        g, p = self.g, self.p
        x0, y0 = p["x0"], p["y0"]
        Uan = ocp(self.U[ANODE], x0)
        Uca = 0.0 if self.half else ocp(self.U[CATHODE], y0)   # Li foil: eta = Phi - phi_e (Sec. 2.2)
        c = np.where(g.lab == PORE, p["c0"],
                     np.where(g.lab == ANODE, x0 * p["cmax_an"], y0 * p["cmax_ca"])).astype(float)
        phi = np.where(g.lab == PORE, -Uan, np.where(g.lab == ANODE, 0.0, Uca - Uan)).astype(float)
        # i_pl = 0 at phi_s - phi_e = U_an  <=>  f_pre(n) = exp(-F U_an / RT)
        f = np.exp(-FARADAY * Uan / self.RT)
        n_eq = p["n_c"] * (f / (1.0 - f)) ** 0.25
        n = np.full(g.F_pl, n_eq)
        return np.concatenate([c, phi, n])

    def split(self, u):
        N = self.N
        return u[:N], u[N:2 * N], u[2 * N:]

    # ------------------------------------------------------------- kinetics
    def interface_currents(self, u):
        """Per interface face: intercalation current i_int (eq. 2.5; on the
        Li foil of a half cell the counter-electrode law 2 i00_ce
        sinh(F eta / 2RT) with eta = Phi - phi_e) and, on anode faces with
        plating on, plating current i_pl (eq. 2.8).  Positive = current from
        solid into electrolyte."""
        g = self.g
        c, phi, n = self.split(u)
        cs, ce = c[g.if_s], c[g.if_p]
        ps, pe = phi[g.if_s], phi[g.if_p]
        ph = g.if_phase
        cmax = np.where(ph == ANODE, self.cmax[ANODE], self.cmax[CATHODE])
        x = cs / cmax
        U = np.where(ph == ANODE, ocp(self.U[ANODE], x), ocp(self.U[CATHODE], x))
        i00 = np.where(ph == ANODE, self.i00[ANODE], self.i00[CATHODE])
        eta = ps - U - pe
        i_int = 2.0 * i00 * np.sqrt(cs * ce) * np.sinh(self.beta * eta)
        if self.half:
            foil = ph == CATHODE
            i_int[foil] = 2.0 * self.p["i00_ce"] * np.sinh(self.beta * (ps[foil] - pe[foil]))
        i_pl = np.zeros(g.F_if)
        if self.p["plating"] and g.F_pl:
            f = g.pl_face
            a = self.beta * (ps[f] - pe[f])
            i_pl[f] = self.p["i00_pl"] * np.sqrt(ce[f]) * (f_pre(n, self.p["n_c"]) * np.exp(a) - np.exp(-a))
        return i_int, i_pl

    # ------------------------------------------------------------- residual
    def residual(self, u, u_old, dt):
        g, p = self.g, self.p
        A, V, h = self.A, self.V, self.h
        c, phi, n = self.split(u)
        c_old, _, n_old = self.split(u_old)
        Rc = V * (c - c_old) / dt
        Rp = np.zeros(self.N)
        # pore-pore faces, eqs. (2.3)-(2.4): j = -kappa grad phi + kappa (1-t+) theta RT/F grad ln c
        a, b = g.pp_lo, g.pp_hi
        j = (-p["kappa"] * (phi[b] - phi[a]) / h
             + p["kappa"] * (1.0 - p["tplus"]) * p["thermo"] * self.RT / FARADAY
             * (np.log(c[b]) - np.log(c[a])) / h)
        Nf = -p["De"] * (c[b] - c[a]) / h + p["tplus"] / FARADAY * j
        np.add.at(Rc, a, A * Nf)
        np.add.at(Rc, b, -A * Nf)
        np.add.at(Rp, a, A * j)
        np.add.at(Rp, b, -A * j)
        # solid-solid faces, eqs. (2.1)-(2.2)
        a, b = g.ss_lo, g.ss_hi
        Ds = np.where(g.ss_phase == ANODE, self.Ds[ANODE], self.Ds[CATHODE])
        sg = np.where(g.ss_phase == ANODE, self.sig[ANODE], self.sig[CATHODE])
        Nf = -Ds * (c[b] - c[a]) / h
        j = -sg * (phi[b] - phi[a]) / h
        np.add.at(Rc, a, A * Nf)
        np.add.at(Rc, b, -A * Nf)
        np.add.at(Rp, a, A * j)
        np.add.at(Rp, b, -A * j)
        # interface faces, eq. (2.4) interface conditions with (2.5) and (2.8)/(2.12)
        i_int, i_pl = self.interface_currents(u)
        # the Li foil carries no concentration equation (Sec. 2.2): no molar flux into it
        solid_mol = np.where(g.if_phase == CATHODE, 0.0, i_int) if self.half else i_int
        np.add.at(Rc, g.if_s, A * solid_mol / FARADAY)
        np.add.at(Rp, g.if_s, A * (i_int + i_pl))
        np.add.at(Rc, g.if_p, -A * (i_int + i_pl) / FARADAY)
        np.add.at(Rp, g.if_p, -A * (i_int + i_pl))
        # current collectors: anode at phi = 0 across half a voxel; cathode galvanostatic
        Rp[g.bot] += A * p["sigma_an"] * phi[g.bot] / (0.5 * h)
        Rp[g.top] += -p["I_app"] / g.top.size
        Rn = A * (n - n_old) / dt + A * i_pl[g.pl_face] / FARADAY
        return np.concatenate([Rc, Rp, Rn])

    # ------------------------------------------------------------- jacobian
    def jacobian(self, u, dt):
        """Analytic dF/du as a CSR matrix."""
        g, p = self.g, self.p
        A, V, h, N = self.A, self.V, self.h, self.N
        c, phi, n = self.split(u)
        rows, cols, vals = [], [], []

        def add(r, cidx, v):
            rows.append(np.asarray(r))
            cols.append(np.asarray(cidx))
            vals.append(np.broadcast_to(np.asarray(v, dtype=float), np.shape(r)).copy())

        iC = lambda i: i          # noqa: E731  concentration unknown / row
        iP = lambda i: N + i      # noqa: E731  potential unknown / row
        vox = np.arange(N)
        add(iC(vox), iC(vox), V / dt)

        # pore-pore
        a, b = g.pp_lo, g.pp_hi
        K = p["kappa"] * (1.0 - p["tplus"]) * p["thermo"] * self.RT / FARADAY / h
        dj = [("p", a, p["kappa"] / h, 0.0), ("p", b, -p["kappa"] / h, 0.0),
              ("c", a, -K / c[a], p["De"] / h), ("c", b, K / c[b], -p["De"] / h)]
        for var, w, dv, ddiff in dj:
            col = iC(w) if var == "c" else iP(w)
            dN = p["tplus"] / FARADAY * dv + ddiff
            add(iC(a), col, A * dN)
            add(iC(b), col, -A * dN)
            add(iP(a), col, A * dv)
            add(iP(b), col, -A * dv)

        # solid-solid
        a, b = g.ss_lo, g.ss_hi
        Ds = np.where(g.ss_phase == ANODE, self.Ds[ANODE], self.Ds[CATHODE])
        sg = np.where(g.ss_phase == ANODE, self.sig[ANODE], self.sig[CATHODE])
        for w, sgn in ((a, 1.0), (b, -1.0)):
            add(iC(a), iC(w), A * sgn * Ds / h)
            add(iC(b), iC(w), -A * sgn * Ds / h)
            add(iP(a), iP(w), A * sgn * sg / h)
            add(iP(b), iP(w), -A * sgn * sg / h)

        # interface: i_int(cs, ce, ps, pe)
        s, e, ph = g.if_s, g.if_p, g.if_phase
        cs, ce, ps, pe = c[s], c[e], phi[s], phi[e]
        cmax = np.where(ph == ANODE, self.cmax[ANODE], self.cmax[CATHODE])
        x = cs / cmax
        Ua = np.where(ph == ANODE, 1, 0)
        U = np.where(Ua == 1, ocp(self.U[ANODE], x), ocp(self.U[CATHODE], x))
        dU = np.where(Ua == 1, docp(self.U[ANODE], x), docp(self.U[CATHODE], x)) / cmax
        i00 = np.where(ph == ANODE, self.i00[ANODE], self.i00[CATHODE])
        eta = ps - U - pe
        pre = 2.0 * i00 * np.sqrt(cs * ce)
        i_int = pre * np.sinh(self.beta * eta)
        gcond = pre * self.beta * np.cosh(self.beta * eta)
        d_cs, d_ce = i_int / (2 * cs) - gcond * dU, i_int / (2 * ce)
        mol_s = np.ones(s.size)                    # share of the face's molar flux in the solid's c row
        if self.half:
            foil = ph == CATHODE
            ef = ps[foil] - pe[foil]
            i_int[foil] = 2.0 * p["i00_ce"] * np.sinh(self.beta * ef)
            gcond[foil] = 2.0 * p["i00_ce"] * self.beta * np.cosh(self.beta * ef)
            d_cs[foil] = 0.0
            d_ce[foil] = 0.0
            mol_s[foil] = 0.0
        d_int = [(iC(s), d_cs), (iC(e), d_ce), (iP(s), gcond), (iP(e), -gcond)]
        for col, dv in d_int:
            add(iC(s), col, A * dv * mol_s / FARADAY)
            add(iP(s), col, A * dv)
            add(iC(e), col, -A * dv / FARADAY)
            add(iP(e), col, -A * dv)

        # plating on anode faces: i_pl(ce, ps, pe, n)
        fpl = g.pl_face
        rn = 2 * N + np.arange(g.F_pl)
        add(rn, rn, A / dt)
        if p["plating"] and g.F_pl:
            s, e = g.if_s[fpl], g.if_p[fpl]
            a_ = self.beta * (phi[s] - phi[e])
            sq = np.sqrt(c[e])
            fp = f_pre(n, p["n_c"])
            ip = p["i00_pl"] * sq * (fp * np.exp(a_) - np.exp(-a_))
            gp = p["i00_pl"] * sq * self.beta * (fp * np.exp(a_) + np.exp(-a_))
            d_pl = [(iC(e), ip / (2 * c[e])), (iP(s), gp), (iP(e), -gp),
                    (rn, p["i00_pl"] * sq * np.exp(a_) * df_pre(n, p["n_c"]))]
            for cc, dv in d_pl:
                add(iP(s), cc, A * dv)
                add(iC(e), cc, -A * dv / FARADAY)
                add(iP(e), cc, -A * dv)
                add(rn, cc, A * dv / FARADAY)

        # anode collector
        add(iP(g.bot), iP(g.bot), A * p["sigma_an"] / (0.5 * h))
        M = self.n_unknowns
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(M, M))

    # ------------------------------------------------------------- scaling
    def scaled_residual(self, R, dt):
        """Dimensionless residual: R^c as a relative concentration change per
        step, R^p relative to the applied current density, R^n relative to n_c."""
        N = self.N
        rc = R[:N] * dt / (self.V * self.c_ref)
        rp = R[N:2 * N] / (self.A * self.mu_ref)
        rn = R[2 * N:] * dt / (self.A * self.p["n_c"])
        return np.concatenate([rc, rp, rn])

    def scaled_update(self, du):
        N = self.N
        return np.concatenate([du[:N] / self.c_ref, du[N:2 * N] * FARADAY / self.RT,
                               du[2 * N:] / self.p["n_c"]])

    def feasible(self, u):
        c, _, n = self.split(u)
        g = self.g
        if np.any(c <= 0.0) or not np.all(np.isfinite(u)):
            return False
        cs = c[g.lab != PORE]
        cm = self.c_ref[g.lab != PORE]
        return bool(np.all(cs < cm) and np.all(n >= 0.0))

    # ------------------------------------------------------------- outputs
    def voltage(self, u):
        """Cell voltage s_cp: mean potential of the cathode collector plane,
        extrapolated from the top cathode voxels across half a voxel."""
        g, p = self.g, self.p
        _, phi, _ = self.split(u)
        j_out = -p["I_app"] / (g.top.size * self.A)
        return float(np.mean(phi[g.top] - j_out * self.h / (2.0 * p["sigma_ca"])))

    def inventories(self, u):
        """Li amounts (mol): electrolyte, anode solid, cathode solid, plated."""
        g = self.g
        c, _, n = self.split(u)
        V = self.V
        return {"electrolyte": float(np.sum(c[g.lab == PORE]) * V),
                "anode": float(np.sum(c[g.lab == ANODE]) * V),
                "cathode": float(np.sum(c[g.lab == CATHODE]) * V),
                "plated": float(np.sum(n) * self.A)}

    def mean_solid(self, u):
        """s_ac: mean Li concentration in each electrode's solid."""
        g = self.g
        c = u[:self.N]
        return {"anode": float(np.mean(c[g.lab == ANODE])), "cathode": float(np.mean(c[g.lab == CATHODE]))}


class NewtonFailure(RuntimeError):
    pass


def lu_solve(J, r):
    """Solve J x = r by SuperLU after scaling each row by its largest entry
    (the rows mix mol/s and A, which would otherwise mislead pivoting)."""
    d = 1.0 / np.asarray(abs(J).max(axis=1).todense()).ravel()
    Js = sp.diags(d) @ J
    return spla.splu(Js.tocsc()).solve(d * r)


def newton_step(model: Model, u_old, dt, u_guess=None, tol_du=1e-10, tol_res=1e-6,
                max_iter=50, max_halvings=20, solve=None):
    """One implicit Euler step: damped Newton on F(u; u_old) = 0.

    Each iteration solves J du = -F by sparse LU (SuperLU), then halves the
    step until the state stays admissible (c > 0, c_s < c_max, n >= 0) and the
    scaled 2-norm residual does not grow.  Converged when the scaled update
    max|du| <= tol_du and the scaled residual max-norm <= tol_res.
    Returns (u_new, info); raises NewtonFailure otherwise.
    """
    if solve is None:
        solve = lu_solve
    u = np.array(u_old if u_guess is None else u_guess, dtype=float)
    R = model.residual(u, u_old, dt)
    r0 = float(np.max(np.abs(model.scaled_residual(R, dt))))
    hist = []
    for it in range(1, max_iter + 1):
        J = model.jacobian(u, dt)
        du = -solve(J, R)
        nrm = np.linalg.norm(model.scaled_residual(R, dt))
        lam = 1.0
        for _ in range(max_halvings + 1):
            u_try = u + lam * du
            if model.feasible(u_try):
                R_try = model.residual(u_try, u_old, dt)
                n_try = np.linalg.norm(model.scaled_residual(R_try, dt))
                if n_try <= nrm or n_try <= 1e-8 * np.sqrt(R.size) or lam < 2 ** -max_halvings:
                    break
            lam *= 0.5
        else:
            raise NewtonFailure("line search failed")
        u, R = u_try, R_try
        step = float(np.max(np.abs(model.scaled_update(lam * du))))
        res = float(np.max(np.abs(model.scaled_residual(R, dt))))
        hist.append((lam, step, res))
        if step <= tol_du and res <= tol_res:
            return u, {"newton_iters": it, "res0": r0, "res_final": res, "history": hist}
    raise NewtonFailure(f"no convergence in {max_iter} iterations: {hist[-3:]}")


def cutoff_reached(V: float, V_cut, I_app: float) -> bool:
    """Voltage cutoff of a constant-current run: a charge (I_app >= 0) stops
    once the cell voltage is at or above V_cut, a discharge once it is at or
    below it.  No interpolation inside a step: the step that crosses is the
    last one."""
    if V_cut is None or V_cut <= 0:
        return False
    return V >= V_cut if I_app >= 0 else V <= V_cut


def simulate(labels, prm: dict, dt: float, steps: int, u0=None, V_cut=None, **kw):
    """Run up to `steps` implicit Euler steps from the equilibrium (or u0),
    stopping after the first step whose cell voltage reaches V_cut (if given).
    Returns the model, the list of states [u^0, ..., u^k] and per-step infos."""
    model = Model(Geometry(labels), prm)
    u = model.initial_state() if u0 is None else np.array(u0, dtype=float)
    states = [u]
    infos = []
    for _ in range(steps):
        u, info = newton_step(model, u, dt, **kw)
        states.append(u)
        infos.append(info)
        if cutoff_reached(model.voltage(u), V_cut, prm["I_app"]):
            break
    return model, states, infos


def lte_estimate(model: Model, u_new, u_old, u_prev, dt, dt_prev) -> float:
    """Local-error estimate of an implicit Euler step (reading R-5 of the
    adaptive stepping of Sec. 2.4).  On an implicit Euler trajectory the
    backward difference (u_old - u_prev)/dt_prev is exactly the time
    derivative the previous step solved for at u_old, so the linear
    extrapolation
        u_pred = u_old + (dt/dt_prev) (u_old - u_prev)
    is the explicit Euler step from u_old.  The two Euler steps carry local
    errors of +-(dt^2/2) u'', hence the implicit step's local error is
        |u_new - u_pred| / 2
    to leading order, whatever dt_prev.  Only the unknowns with a time
    derivative enter: the concentrations, relative to c0 / c_max, and the
    plated amounts, relative to n_c.  The potentials are algebraic (charge
    conservation holds at every instant, so they jump with the applied
    current) and carry no truncation error of their own."""
    N = model.N
    w = dt / dt_prev
    c = u_new[:N] - (u_old[:N] + w * (u_old[:N] - u_prev[:N]))
    n = u_new[2 * N:] - (u_old[2 * N:] + w * (u_old[2 * N:] - u_prev[2 * N:]))
    e = np.abs(c) / model.c_ref
    if n.size:
        e = np.concatenate([e, np.abs(n) / model.p["n_c"]])
    return float(0.5 * np.max(e))


def simulate_adaptive(labels, prm: dict, t_end: float, dt0: float, dt_min: float, dt_max: float, tol: float,
                      max_steps: int = 10000, **kw):
    """Adaptive implicit Euler from the equilibrium to t_end (reading R-5).

    Step sizes change by factors of 2 only: a step whose Newton iteration
    fails, or whose error estimate exceeds tol, is rejected and redone with
    half the step (failure below dt_min); an accepted step whose estimate is
    at most tol/4 doubles the next step (at most dt_max); a step that would
    pass t_end is shortened to end there.  The first step has no estimate.
    Returns the model, the accepted times, states and step sizes, the
    estimates of the accepted steps and the number of rejected steps."""
    model = Model(Geometry(labels), prm)
    u = model.initial_state()
    t, dt, dt_prev, u_prev = 0.0, dt0, None, None
    times, states, dts, ests = [0.0], [u], [], []
    rejected = 0
    while t < t_end and len(dts) < max_steps:
        h = min(dt, t_end - t)
        try:
            u_new, _ = newton_step(model, u, h, **kw)
            est = None if u_prev is None else lte_estimate(model, u_new, u, u_prev, h, dt_prev)
        except NewtonFailure:
            u_new, est = None, np.inf
        if u_new is None or (est is not None and est > tol):
            rejected += 1
            dt = h / 2.0
            if dt < dt_min:
                raise NewtonFailure(f"adaptive step below dt_min at t = {t}")
            continue
        u_prev, u, dt_prev = u, u_new, h
        t = t + h if t + h < t_end else t_end
        times.append(t)
        states.append(u)
        dts.append(h)
        ests.append(est)
        dt = min(2.0 * h, dt_max) if (est is not None and est <= tol / 4.0) else h
    return model, times, states, dts, ests, rejected
