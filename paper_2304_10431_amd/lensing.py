"""Lensing operator built on the general SHT (Sect. 2 and the end of Sect. 3).

The lensed field at the points n_i is the unlensed field synthesised at the
deflected points n'_i, with the spin phase e^{i s chi} for spin s > 0 (eq. forwardpol);
the deflection field is the spin-1 synthesis of sqrt(L (L+1)) (phi_LM + i Omega_LM)
on the points n_i (eq. deflect).  ``Lensing`` builds both plans once (positions
are fixed per instance, as when many maps share one set of angles) and offers the
forward operator, its adjoint, and the gradients of a real loss of the lensed map
with respect to the unlensed coefficients and to the lensing potentials.

Every step runs in the library: spin-1 synthesis, ``gsht_alm_lscale``,
``gsht_deflect``, the plan at the deflected points, ``gsht_spin_phase`` and, for
gradients, ``gsht_spin_phase_vjp``, ``gsht_plan_synth_vjp`` and ``gsht_deflect_vjp``.
"""
from __future__ import annotations

import torch

from . import gsht


def deflected_points(theta, phi, plm, lmax_p: int, mmax_p: int | None = None,
                     epsilon: float = 1e-13):
    """The points n' that the lensing potential plm (band limits lmax_p, mmax_p) maps
    theta, phi to: the deflection is the FP64 gradient-only spin-1 synthesis of
    sqrt(L (L+1)) phi_LM at the points (eq. deflect), then the great-circle step
    (``gsht_deflect``).  Returns (theta', phi') as FP64 device tensors."""
    mmax_p = lmax_p if mmax_p is None else mmax_p
    plan = gsht.Plan(theta, phi, lmax_p, mmax_p, 1, epsilon, "f64")
    try:
        glm = gsht.alm_lscale(plm.to(torch.complex128).reshape(1, -1).contiguous(), lmax_p, mmax_p)
        alpha = plan.synth_grad(glm)
    finally:
        plan.close()
    th, ph, _ = gsht.deflect(theta, phi, alpha, want_chi=False)
    return th, ph


class Lensing:
    """D_alpha for one geometry: points (theta, phi), lensing potential plm (and curl
    potential olm) with band limits (lmax_p, mmax_p), unlensed field band limits
    (lmax, mmax), spin, accuracy epsilon and precision.  sigma is the oversampling
    choice of both plans (None: 2; 2, 1.5 or 1.25; "tuned": the fastest by timing)."""

    def __init__(self, theta, phi, plm, lmax: int, mmax: int, spin: int, epsilon: float,
                 precision="f64", olm=None, lmax_p: int | None = None, mmax_p: int | None = None,
                 sigma=None):
        self.spin = spin
        self.lmax_p = lmax if lmax_p is None else lmax_p
        self.mmax_p = self.lmax_p if mmax_p is None else mmax_p
        prec = gsht._PREC[precision]
        cdt = gsht._CDT[prec]
        self.theta = theta
        self.phi = phi
        self.dplan = gsht.Plan(theta, phi, self.lmax_p, self.mmax_p, 1, epsilon, precision,
                               sigma=sigma)
        if olm is None:   # no curl potential: gradient-only spin-1 synthesis
            glm = gsht.alm_lscale(plm.to(cdt).reshape(1, -1).contiguous(), self.lmax_p, self.mmax_p)
            self.alpha = self.dplan.synth_grad(glm)
        else:
            glm = torch.stack([plm.to(cdt), olm.to(cdt)]).contiguous()
            glm = gsht.alm_lscale(glm, self.lmax_p, self.mmax_p)
            self.alpha = self.dplan.synth(glm)
        self._pot = (plm.to(cdt), None if olm is None else olm.to(cdt), epsilon, precision)
        self.theta_d, self.phi_d, chi = gsht.deflect(theta, phi, self.alpha, want_chi=spin > 0)
        self.chi = chi
        self.plan = gsht.Plan(self.theta_d, self.phi_d, lmax, mmax, spin, epsilon, precision,
                              sigma=sigma)

    def close(self):
        self.plan.close()
        self.dplan.close()

    def update(self, plm, olm=None):
        """New lensing potential (and curl potential) on the same points: the deflection
        is resynthesised and the lensed plan moved to the new deflected points
        (gsht_plan_set_points), without building new plans."""
        _, olm_, eps, prec = self._pot
        cdt = gsht._CDT[gsht._PREC[prec]]
        if (olm is None) != (olm_ is None):
            raise ValueError("update must keep the same potentials (curl given or not)")
        if olm is None:
            glm = gsht.alm_lscale(plm.to(cdt).reshape(1, -1).contiguous(), self.lmax_p, self.mmax_p)
            alpha = self.dplan.synth_grad(glm)
        else:
            glm = gsht.alm_lscale(torch.stack([plm.to(cdt), olm.to(cdt)]).contiguous(),
                                  self.lmax_p, self.mmax_p)
            alpha = self.dplan.synth(glm)
        theta_d, phi_d, chi = gsht.deflect(self.theta, self.phi, alpha, want_chi=self.spin > 0)
        # the operator's state changes only once the plan has accepted the new points
        self.plan.set_points(theta_d, phi_d)
        self.alpha, self.theta_d, self.phi_d, self.chi = alpha, theta_d, phi_d, chi
        self._pot = (plm.to(cdt), None if olm is None else olm.to(cdt), eps, prec)

    def forward(self, alm):
        """Lensed map [ncomp][npts]."""
        m = self.plan.synth(alm)
        if self.spin:
            gsht.spin_phase(m, self.chi, self.spin, 1)
        return m

    def adjoint(self, maps):
        """Adjoint of ``forward`` (eq. adjoint and its spin-s form): a_lm [ncomp][nalm]."""
        if self.spin:
            maps = gsht.spin_phase(maps.clone(), self.chi, self.spin, -1)
        return self.plan.adjoint(maps)

    def magnification(self):
        """|A| at the points (Appendix B): convergence kappa (+ rotation omega) by a spin-0
        synthesis of l(l+1)/2 (phi_LM, Omega_LM), shear by a spin-2 synthesis of
        sqrt((l-1)l(l+1)(l+2))/2 (phi_LM, Omega_LM), then gsht_magnification."""
        plm, olm, eps, prec = self._pot
        lp, mp = self.lmax_p, self.mmax_p
        p0 = gsht.Plan(self.theta, self.phi, lp, mp, 0, eps, prec)
        p2 = gsht.Plan(self.theta, self.phi, lp, mp, 2, eps, prec)
        kappa = p0.synth(gsht.alm_lfactor(plm.reshape(1, -1).contiguous(), lp, mp, 1))
        omega = None
        if olm is not None:
            omega = p0.synth(gsht.alm_lfactor(olm.reshape(1, -1).contiguous(), lp, mp, 1))
            gam = p2.synth(gsht.alm_lfactor(torch.stack([plm, olm]).contiguous(), lp, mp, 2))
        else:
            gam = p2.synth_grad(gsht.alm_lfactor(plm.reshape(1, -1).contiguous(), lp, mp, 2))
        det = gsht.magnification(self.alpha, kappa, gam, omega)
        p0.close()
        p2.close()
        return det

    def inverse(self, maps, weights):
        """Approximate inverse lensing (Appendix B): the adjoint applied to the lensed map
        times the quadrature weights and the magnification determinant."""
        w = gsht.map_weight(self.magnification().reshape(1, -1), weights).reshape(-1)
        return self.adjoint(gsht.map_weight(maps, w))

    def vjp(self, alm, gmap, want_alm=True, want_potential=True):
        """Gradients of a real loss L with dL/dmap = gmap (torch's convention for complex
        tensors): (dL/dalm, dL/dplm, dL/dolm); entries not asked for are None."""
        g_unrot, g_chi = gmap, None
        if self.spin:
            lensed = self.forward(alm) if want_potential else None
            g_unrot, g_chi = gsht.spin_phase_vjp(gmap, lensed, self.chi, self.spin,
                                                 want_chi=want_potential)
        galm, gth, gph = self.plan.synth_vjp(alm, g_unrot, want_alm, want_potential, want_potential)
        if not want_potential:
            return galm, None, None
        g_alpha = gsht.deflect_vjp(self.theta, self.alpha, gth, gph, g_chi)
        gg, _, _ = self.dplan.synth_vjp(None, g_alpha, True, False, False)
        gp = gsht.alm_lscale(gg, self.lmax_p, self.mmax_p)
        return galm, gp[0], gp[1]


class LensedAlm:
    """Lensed coefficients from unlensed ones (Sect. 4): the lensed map on a grid with
    quadrature weights (e.g. Gauss-Legendre), then the weighted adjoint synthesis
    (a standard analysis) up to (lmax_len, mmax_len); ``adjoint`` is the exact
    adjoint of the whole chain (synthesis on the grid, weights, lensing adjoint)."""

    def __init__(self, theta, phi, weights, plm, lmax: int, mmax: int, lmax_len: int,
                 mmax_len: int, spin: int, epsilon: float, precision="f64", olm=None,
                 lmax_p: int | None = None, mmax_p: int | None = None):
        self.lens = Lensing(theta, phi, plm, lmax, mmax, spin, epsilon, precision, olm=olm,
                            lmax_p=lmax_p, mmax_p=mmax_p)
        self.weights = weights
        self.ana = gsht.Plan(theta, phi, lmax_len, mmax_len, spin, epsilon, precision)

    def close(self):
        self.lens.close()
        self.ana.close()

    def forward(self, alm):
        m = self.lens.forward(alm)
        return self.ana.adjoint(gsht.map_weight(m, self.weights, out=m))

    def adjoint(self, alm_len):
        m = self.ana.synth(alm_len)
        return self.lens.adjoint(gsht.map_weight(m, self.weights, out=m))
