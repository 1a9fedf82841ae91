"""Pins of the oracle's Potthoff functional (oracle/vca.py) on the CPU:

  * the analytic pole formula (eq. (omega4)) equals the numerical frequency
    integral of eq. (sef4) along the imaginary axis (an independent route:
    quadrature of ln det[1 - V G'(i w)]), on the 2x2 plaquette at U = 8 and
    on the 4-site chain at U = 4, for several reference hoppings;
  * at U = 0 the functional is exact for any reference system: it equals
    the free lattice grand potential per cluster (negative one-body energies
    of the lattice's k-dependent matrix) whatever the reference hopping;
  * the Lehmann representation of the reference system satisfies
    Q Q^T = 1 (both parts).
"""
import numpy as np
import pytest

import synth
from oracle import vca as O


@pytest.mark.parametrize("s,nk", [(synth.vca_plaquette(tp=-1.2), 4),
                                  (synth.vca_plaquette(tp=-0.8), 4),
                                  (synth.vca_chain4(tp=-1.1), 8)],
                         ids=["plaq_tp1.2", "plaq_tp0.8", "chain4_tp1.1"])
def test_pole_formula_equals_numeric_integral(s, nk):
    e0, poles, Q = O.cluster_lehmann(s.t_ref, s.U, s.nup, s.ndn)
    assert np.abs(Q @ Q.T - np.eye(Q.shape[0])).max() <= 1e-12
    ks = synth.k_grid_2d(nk) if "plaq" in s.name else synth.k_grid_1d(nk)
    a = O.omega_poles(e0, poles, Q, s.dt, s.bonds, ks)
    b = O.omega_numeric(e0, poles, Q, s.dt, s.bonds, ks)
    assert abs(a - b) <= 1e-8 * max(1.0, abs(a))


@pytest.mark.parametrize("tp", [-0.7, -1.0, -1.3])
def test_noninteracting_functional_is_exact(tp):
    s = synth.vca_chain4(U=0.0, mu=0.0, tp=tp)
    e0, poles, Q = O.cluster_lehmann(s.t_ref, s.U, s.nup, s.ndn)
    ks = synth.k_grid_1d(32)
    a = O.omega_poles(e0, poles, Q, s.dt, s.bonds, ks)
    assert abs(a - O.omega_free(s.h0, s.bonds, ks)) <= 1e-10
