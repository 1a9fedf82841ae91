"""The Potthoff functional on the GPU against the oracle (oracle/vca.py):

  * from the same Lehmann form (the oracle's exhausted band Lanczos), the
    pole-formula functional and its per-k sums, relative 1e-12;
  * the whole path (GPU ground state, GPU band Lanczos to exhaustion, GPU k
    sum) against the oracle's pole formula, 1e-9, on the 2x2 plaquette at
    U = 8 for three reference hoppings;
  * at U = 0 the functional equals the free lattice grand potential per
    cluster for any reference hopping (4-site chain), 1e-9.
"""
import numpy as np
import pytest

import synth
from oracle import vca as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2305_18643_amd as q
    return q


def test_vca_omega_matches_oracle(q):
    s = synth.vca_plaquette(tp=-1.2)
    e0, poles, Q = O.cluster_lehmann(s.t_ref, s.U, s.nup, s.ndn)
    ks = synth.k_grid_2d(8)
    om, per = q.vca_omega(e0, poles, Q, s.dt, s.bonds, ks)
    ref = O.omega_poles(e0, poles, Q, s.dt, s.bonds, ks)
    for i, k in enumerate(ks):
        Lk = np.diag(poles) + Q.T @ O.v_of_k(4, s.dt, s.bonds, k) @ Q
        w = np.linalg.eigvalsh(0.5 * (Lk + Lk.conj().T))
        assert abs(per[i] - w[w < 0].sum()) <= 1e-12 * max(1.0, abs(per[i]))
    print(f"  vca omega {om:.12f} (oracle {ref:.12f}), R = {len(poles)}")
    assert abs(om - ref) <= 1e-12 * abs(ref)


@pytest.mark.parametrize("tp", [-0.8, -1.0, -1.3])
def test_vca_full_path_matches_oracle(q, tp):
    s = synth.vca_plaquette(tp=tp)
    ks = synth.k_grid_2d(16)
    om = q.vca.omega(s, ks)
    e0, poles, Q = O.cluster_lehmann(s.t_ref, s.U, s.nup, s.ndn)
    ref = O.omega_poles(e0, poles, Q, s.dt, s.bonds, ks)
    print(f"  vca plaquette tp={tp}: omega {om:.12f} (oracle {ref:.12f})")
    assert abs(om - ref) <= 1e-9 * abs(ref)


@pytest.mark.parametrize("tp", [-0.7, -1.3])
def test_vca_noninteracting_is_exact(q, tp):
    s = synth.vca_chain4(U=0.0, mu=0.0, tp=tp)
    ks = synth.k_grid_1d(32)
    om = q.vca.omega(s, ks)
    ref = O.omega_free(s.h0, s.bonds, ks)
    print(f"  vca chain4 U=0 tp={tp}: omega {om:.12f}, exact {ref:.12f}")
    assert abs(om - ref) <= 1e-9 * max(1.0, abs(ref))
