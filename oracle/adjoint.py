"""FP64 discrete adjoint of the oracle's time step.

TEST INFRASTRUCTURE ONLY (like oracle/kspace.py): it is the reference the
HIP adjoint is compared with, and it is itself pinned by finite differences
of the FP64 forward model in the tests.

Objective.  The recorded intensity I(x) = (1/N_w) sum_m p^m(x)^2 / (rho0 c0)(x)
over the steps m >= record_start (time-mean intensity, Section 5 records
aggregate quantities of this kind), and J = sum_x w(x) I(x) for a weight map
w (for the focusing objective: +1/|S_in| inside a sphere at the focus and
-1/|S_out| at the other non-PML points).  The parameters are the amplitude a_e
and phase phi_e of every source element, s_e(n) = a_e sin(omega (n+1/2) dt +
phi_e).

Reverse pass.  Step n maps (p^n, u^(n-1/2), rho_xi^n) to
(p^(n+1), u^(n+1/2), rho_xi^(n+1)) through Eqs. (4a)-(4d), (6), (8) exactly as
in Oracle._one_step.  Its transpose, applied to the adjoints
(pb, ub_xi, rb_xi) of the step's outputs, is taken line by line in reverse:
  * a spectral operator f -> IFT(m FT f) with m(-k) = conj m(k) is a real
    linear map whose transpose is f -> IFT(conj(m) FT f); so the adjoint of
    the gradient (m = D+ kappa) multiplies by conj(D+ kappa), that of the
    divergence by conj(D- kappa), and the absorption operators (real, even
    k^(y-2), k^(y-1)) are their own transposes;
  * Eq. (6):  p = c0^2 (rho + B/(2A rho0) rho^2 + tau a - eta b):
        rb_total = c0^2 (1 + B/A rho / rho0) pb,  ab = c0^2 tau pb,  bb = -c0^2 eta pb;
  * Eq. (8):  a = IFT(k^(y-2) FT(rho0 sum d)),  b = IFT(k^(y-1) FT(rho)):
        db_xi += rho0 IFT(k^(y-2) FT ab),  rb_total += IFT(k^(y-1) FT bb);
  * Eq. (4d): rho_xi' = q (q rho_xi - dt rho0 d_xi) / (1 + 2 dt d_xi) + src:
        R_xi = rb_xi + rb_total,  rb_xi <- R_xi q^2 / den,
        db_xi += -R_xi (q dt rho0 + 2 dt (rho_xi' - src)) / den,
        dJ/ds_e(n) = sum over the element's points of dt coef R_xi summed over xi;
  * Eq. (4b): u' = q+ (q+ u - dt / rho0+ g):  gb_xi = -q+ dt / rho0+ ub_xi,  ub <- q+^2 ub;
  * loss: pb += 2 w p^m / (rho0 c0 N_w) for every recorded step m.
Finally dJ/da_e = sum_n dJ/ds_e(n) sin(theta_n), dJ/dphi_e = sum_n dJ/ds_e(n) a_e cos(theta_n).
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from .kspace import Oracle


class AdjointOracle:
    def __init__(self, scen, weights, workers: Optional[int] = None):
        self.scen = scen
        self.o = Oracle(scen, workers=workers)
        self.w = np.asarray(weights, np.float64).reshape(self.o.shape)
        self.steps = int(scen.steps)
        self.record_start = int(scen.sensor.record_start)
        self.n_window = self.steps - self.record_start + 1
        if self.n_window < 1:
            raise ValueError("the recording window is empty")
        self.J = None

    def forward(self, progress=None) -> float:
        o = self.o
        o.tape = []
        o.step(self.steps, progress)
        rc = o.rho0 * o.c0
        J = 0.0
        for t in o.tape:
            if t["n"] + 1 >= self.record_start:
                J += float(np.sum(self.w * t["p"] ** 2 / rc))
        self.J = J / self.n_window
        return self.J

    def _op(self, m, f):
        o = self.o
        return o.ift(m * o.ft(f))

    def backward(self, progress=None) -> dict:
        """progress(k), if given, is called after the k-th reverse step."""
        o = self.o
        if self.J is None:
            self.forward()
        dt = o.dt
        shape = o.shape
        rc = o.rho0 * o.c0
        c2 = o.c0 ** 2
        pb = np.zeros(shape)
        ub = [np.zeros(shape) for _ in range(3)]
        rb = [np.zeros(shape) for _ in range(3)]
        src = o.src
        ne = len(src["amp"])
        dJds = np.zeros((self.steps, ne))
        for t in reversed(o.tape):
            n = t["n"]
            if n + 1 >= self.record_start:
                pb = pb + 2.0 * self.w * t["p"] / (rc * self.n_window)
            rho = t["rho"]
            # Eq. (6)
            if o.nonlinear:
                rb_tot = c2 * (1.0 + o.bona / o.rho0 * rho) * pb
            else:
                rb_tot = c2 * pb
            db_common = np.zeros(shape)
            if o.absorbing:
                ab = c2 * o.tau * pb
                bb = -c2 * o.eta * pb
                db_common = o.rho0 * self._op(o.k_tau, ab)
                rb_tot = rb_tot + self._op(o.k_eta, bb)
            # Eq. (4d) with the source
            add = np.zeros(o.N)
            np.add.at(add, src["idx"], dt * src["coef"] * o.source_values(n)[src["elem"]])
            add = add.reshape(shape)
            db = []
            R_sum = np.zeros(shape)
            for a in range(3):
                q = o.pml[a]
                R = rb[a] + rb_tot
                R_sum += R
                d = t["div"][a]
                den = 1.0 + 2.0 * dt * d if o.nonlinear else 1.0
                if o.nonlinear:
                    dbar = -R * (q * dt * o.rho0 + 2.0 * dt * (t["rho_parts"][a] - add)) / den
                else:
                    dbar = -R * q * dt * o.rho0
                db.append(dbar + db_common)
                rb[a] = R * q * q / den
            contrib = dt * src["coef"] * R_sum.reshape(-1)[src["idx"]]
            np.add.at(dJds[n], src["elem"], contrib)
            # Eq. (4c): transpose of the divergence
            for a in range(3):
                ub[a] = ub[a] + self._op(np.conj(o.d_minus[a] * o.kappa), db[a])
            # Eq. (4b)
            gb = []
            for a in range(3):
                q = o.pml_stag[a]
                gb.append(-q * dt / o.rho0_stag[a] * ub[a])
                ub[a] = q * q * ub[a]
            # Eq. (4a): transpose of the gradient
            pb = sum(self._op(np.conj(o.d_plus[a] * o.kappa), gb[a]) for a in range(3))
            if progress is not None:
                progress(self.steps - n)
        theta = 2.0 * np.pi * src["freq"] * (np.arange(self.steps) + 0.5) * dt
        ph = theta[:, None] + src["phase"][None, :]
        grad_amp = np.sum(dJds * np.sin(ph), axis=0)
        grad_phase = np.sum(dJds * src["amp"][None, :] * np.cos(ph), axis=0)
        return dict(dJds=dJds, grad_amp=grad_amp, grad_phase=grad_phase)


def objective(scen, weights, workers: Optional[int] = None) -> float:
    """J of one forward run of the FP64 oracle."""
    return AdjointOracle(scen, weights, workers).forward()
