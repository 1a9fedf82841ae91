"""GPU parity: the HIP library through the C ABI against the CPU oracle.

Tolerances:
  * basis, labels: bit-exact;
  * H.v FP64: |dw_i| <= 64 eps (|H| |v|)_i, the rounding bound of a sum of
    at most ~64 products (eps = 2^-53);
  * H.v FP32-vector: FP64 sums rounded to FP32 once per pass; sectors with
    long rows take two passes (in-row term, then row mixing), so
    |dw_i| <= 2^-24 (|w_i| + (|H| |v|)_i) plus the FP64 bound;
  * E0 (FP64): relative 1e-10; G(omega) at eta = 0.1: absolute 1e-4.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import cf

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -53


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2305_18643_amd as q
    q.load_library()
    return q


def _torch():
    import torch
    return torch


# ---------------------------------------------------------------- basis

BASIS_CASES = [(1, 0, 1), (1, 1, 1), (4, 2, 2), (4, 0, 4), (5, 2, 3), (12, 6, 6), (12, 7, 6),
               (14, 7, 7), (16, 8, 8), (16, 9, 8), (13, 1, 12), (20, 10, 9), (24, 12, 3),
               (32, 1, 2), (32, 3, 31), (31, 2, 30)]


@pytest.mark.parametrize("L,nup,ndn", BASIS_CASES)
def test_basis_bit_exact(q, L, nup, ndn):
    print(f"basis L={L} ({nup},{ndn})", flush=True)
    b = q.sector_basis(L, nup, ndn)
    for spin, N in ((0, nup), (1, ndn)):
        st = b.states(spin).cpu().numpy()
        ref = oracle.sector_states(L, N).astype(np.int64)
        assert np.array_equal(st, ref)
        lo, hi = (x.cpu().numpy().astype(np.int64) for x in b.rank_tables(spin))
        l_lo = (L + 1) // 2
        l_hi = L - l_lo
        m = (1 << l_lo) - 1
        lab = lo[st & m] + hi[(np.array([bin(x).count("1") for x in (st & m)]) << l_hi) | (st >> l_lo)]
        assert np.array_equal(lab, np.arange(st.shape[0]))
    assert b.dim == oracle.binom(L, nup) * oracle.binom(L, ndn)


def test_rank_tables_on_random_strings(q):
    L = 16
    b = q.sector_basis(L, 8, 8)
    lo, hi = (x.cpu().numpy().astype(np.int64) for x in b.rank_tables(0))
    rng = np.random.default_rng(5)
    for x in rng.integers(0, 1 << L, 500):
        x = int(x)
        xl, xh = x & 255, x >> 8
        assert lo[xl] + hi[(bin(xl).count("1") << 8) | xh] == oracle.rank(x)


# ---------------------------------------------------------------- H.v

def _hv_models():
    out = [synth.plaquette_2x2(), synth.two_site(), synth.rect_cluster(2, 4, U=4.0, mu=1.0),
           synth.chain(10, U=4.0, mu=2.0, nup=5, ndn=4),
           synth.random_model(101, 9, 4, 5), synth.random_model(102, 11, 3, 6),
           synth.random_model(103, 10, 5, 5, uniform_U=True),
           synth.cluster_3x4(), synth.rect_cluster(3, 3, U=6.0, mu=3.0, nup=5, ndn=4)]
    rng = np.random.default_rng(18643)
    out += [synth.impurity_model(rng, nb) for nb in (2, 5, 9)]
    out.append(synth.rect_cluster(4, 1, U=3.0, mu=0.0, nup=0, ndn=2))
    out.append(synth.rect_cluster(4, 1, U=3.0, mu=0.0, nup=4, ndn=1))
    # long rows (>= 4096 up strings): the two-pass LDS path
    out.append(synth.rect_cluster(4, 4, U=8.0, mu=4.0, nup=8, ndn=1, name="4x4r"))
    out.append(synth.rect_cluster(5, 3, tp=0.3, U=5.0, mu=2.5, nup=7, ndn=2, name="5x3r"))
    m = synth.random_model(104, 16, 8, 2, density=0.12)
    m.U = np.random.default_rng(104).uniform(0, 8, 16)
    out.append(m)
    return out


@pytest.mark.parametrize("m", _hv_models(), ids=lambda m: f"{m.name}_{m.nup}_{m.ndn}")
@pytest.mark.parametrize("prec", ["fp64", "fp32v"])
def test_hv_elementwise(q, m, prec):
    torch = _torch()
    print(f"hv {m.name} ({m.nup},{m.ndn}) {prec}", flush=True)
    b = q.sector_basis(m.L, m.nup, m.ndn)
    rng = np.random.default_rng(7)
    v = rng.uniform(-1, 1, b.dim)
    if prec == "fp32v":
        v = v.astype(np.float32).astype(np.float64)
    dt = torch.float64 if prec == "fp64" else torch.float32
    vd = torch.tensor(v, dtype=dt, device="cuda")
    w = q.hv(m, b, vd).double().cpu().numpy()
    wo = oracle.hv(m.t, m.U, m.nup, m.ndn, v)
    bound = oracle.hv_abs_bound(m.t, m.U, m.nup, m.ndn, v)
    tol = 64 * EPS * bound + 1e-300
    if prec == "fp32v":
        tol = tol + 2.0 ** -24 * (np.abs(wo) + bound)
    err = np.abs(w - wo)
    assert np.all(err <= tol), (err.max(), np.argmax(err - tol))


def test_hv_4x4_sampled_rows(q):
    """Full 16-site sector (d = 165,636,900), the configuration bench.py times:
    the SplitMix64 vector of seed 1, oracle rows computed one by one."""
    torch = _torch()
    m = synth.cluster_4x4(8.0)
    print("hv 4x4 full sector", flush=True)
    b = q.sector_basis(16, 8, 8)
    v = oracle.start_vector(1, b.dim)
    vd = torch.from_numpy(v).to("cuda")
    w = q.hv(m, b, vd)
    rng = np.random.default_rng(3)
    rows = np.unique(np.concatenate([rng.integers(0, b.dim, 20000), np.arange(64),
                                     np.arange(b.dim - 64, b.dim),
                                     12870 * np.arange(0, 12870, 997) + 12869]))
    wr = w[torch.from_numpy(rows).to("cuda")].cpu().numpy()
    wo = oracle.hv_rows(m.t, m.U, 8, 8, v, rows)
    bound = oracle.hv_abs_bound(m.t, m.U, 8, 8, v, rows)
    assert np.all(np.abs(wr - wo) <= 64 * EPS * bound)
    # FP32-vector storage on the same rows
    v32 = vd.float()
    w32 = q.hv(m, b, v32)
    wr32 = w32[torch.from_numpy(rows).to("cuda")].double().cpu().numpy()
    wo32 = oracle.hv_rows(m.t, m.U, 8, 8, v32.cpu().numpy(), rows)
    assert np.all(np.abs(wr32 - wo32) <= 2.0 ** -24 * (np.abs(wo32) + bound) + 64 * EPS * bound)
    del w, w32, vd, v32


def test_hv_sector_over_2gb_sampled_rows(q):
    """An 18-site 2x9 cluster with next-nearest hops (bond-dependent t) in the
    (5, 9) sector: d = 8,568 x 48,620 = 416,576,160, rows long enough for the
    two-pass product.  The FP64 vector (3.3 GB) is past the 2 GB up to which
    the row-mixing pass reads neighbours through a buffer descriptor, so it
    takes the 64-bit-address form; its FP32 copy (1.7 GB) takes the
    descriptor form.  Oracle rows computed one by one."""
    torch = _torch()
    m = synth.rect_cluster(2, 9, tp=0.3, U=4.0, mu=2.0, nup=5, ndn=9, name="2x9")
    print("hv 2x9 (5,9) sector", flush=True)
    b = q.sector_basis(18, 5, 9)
    assert b.dim == 8568 * 48620 and b.dim * 8 > 2 ** 31 > b.dim * 4
    v = oracle.start_vector(7, b.dim)
    vd = torch.from_numpy(v).to("cuda")
    rng = np.random.default_rng(11)
    rows = np.unique(np.concatenate([rng.integers(0, b.dim, 4000), np.arange(64),
                                     np.arange(b.dim - 64, b.dim)]))
    ri = torch.from_numpy(rows).to("cuda")
    bound = oracle.hv_abs_bound(m.t, m.U, 5, 9, v, rows)
    w = q.hv(m, b, vd)
    wr = w[ri].cpu().numpy()
    del w
    wo = oracle.hv_rows(m.t, m.U, 5, 9, v, rows)
    assert np.all(np.abs(wr - wo) <= 64 * EPS * bound)
    v32 = vd.float()
    del vd
    w32 = q.hv(m, b, v32)
    wr32 = w32[ri].double().cpu().numpy()
    del w32
    v32h = v32.cpu().numpy()
    wo32 = oracle.hv_rows(m.t, m.U, 5, 9, v32h, rows)
    assert np.all(np.abs(wr32 - wo32) <= 2.0 ** -24 * (np.abs(wo32) + bound) + 64 * EPS * bound)
    del v32, v32h


# ---------------------------------------------------------------- ground state

GS_MODELS = [synth.plaquette_2x2(), synth.two_site(U=8.0), synth.rect_cluster(2, 4, U=4.0, mu=2.0),
             synth.chain(10, U=4.0, mu=2.0), synth.random_model(201, 8, 4, 3),
             synth.rect_cluster(3, 3, U=6.0, mu=3.0, nup=5, ndn=4),
             synth.rect_cluster(4, 4, U=8.0, mu=4.0, nup=8, ndn=1, name="4x4r")]


@pytest.mark.parametrize("m", GS_MODELS, ids=lambda m: f"{m.name}_{m.nup}_{m.ndn}")
def test_ground_state_fp64(q, m):
    print(f"gs {m.name}", flush=True)
    b = q.sector_basis(m.L, m.nup, m.ndn)
    r = q.lanczos_gs(m, b)
    ro = oracle.lanczos_gs(m.t, m.U, m.nup, m.ndn, want_vector=True)
    assert r["converged"]
    assert abs(r["e0"] - ro["e0"]) <= 1e-10 * abs(ro["e0"])
    psi = r["psi"].cpu().numpy()
    assert abs(np.linalg.norm(psi) - 1.0) < 1e-12
    assert abs(abs(np.dot(psi, ro["psi"])) - 1.0) < 1e-9
    assert r["true_residual"] < 1e-6
    # the first Lanczos coefficients agree before orthogonality is lost
    k = min(10, r["n_iter"], ro["n_iter"])
    assert np.allclose(r["alpha"][:k], ro["alpha"][:k], rtol=1e-10, atol=1e-10)
    assert np.allclose(r["beta"][:k], ro["beta"][:k], rtol=1e-9, atol=1e-10)


def test_ground_state_fp32v_reports_error(q):
    m = synth.chain(10, U=4.0, mu=2.0)
    b = q.sector_basis(m.L, m.nup, m.ndn)
    ro = oracle.lanczos_gs(m.t, m.U, m.nup, m.ndn)
    r = q.lanczos_gs(m, b, prec="fp32v", reorth=1, tol=1e-7)
    rel = abs(r["e0"] - ro["e0"]) / abs(ro["e0"])
    print(f"FP32-vector E0 relative error {rel:.2e}")
    assert rel < 1e-5


def test_fixed_steps_and_breakdown(q):
    # t = 0: H is diagonal; the Krylov space is exhausted after a few steps
    L = 4
    t = np.diag(np.full(L, -3.0))
    U = np.full(L, 6.0)
    b = q.sector_basis(L, 2, 2)
    r = q.lanczos_gs((t, U), b, fixed_steps=50)
    assert r["breakdown"] and r["n_iter"] < 10
    assert abs(r["e0"] + 12.0) < 1e-12


def test_breakdown_long_rows(q):
    # the same on a long-row sector (16 orbitals, (8, 1): the two-pass step
    # with the deferred update): t = 0 but mu = 3, U = 6, so H has the two
    # eigenvalues -27 and -21 and the Krylov space is exhausted at step 2.
    # The step's dots give |x|^2 only to a few eps <w,w>, far above a
    # vanishing beta; the direct norm pass must take over and stop the chain.
    # FP32 vectors leave a residual of ~1e-7 |w| after the space is exhausted
    # (their storage floors it), so there no breakdown is detected; the steps
    # past exhaustion run on that noise and E0 is checked at the FP32 storage
    # level (relative 1e-6; observed 1.3e-7).
    L = 16
    t = np.diag(np.full(L, -3.0))
    U = np.full(L, 6.0)
    b = q.sector_basis(L, 8, 1)
    r = q.lanczos_gs((t, U), b, fixed_steps=40)
    assert r["breakdown"] and r["n_iter"] <= 3, r["n_iter"]
    assert abs(r["e0"] + 27.0) < 1e-12, r["e0"]
    r = q.lanczos_gs((t, U), b, fixed_steps=40, prec="fp32v", reorth=1)
    assert abs(r["e0"] + 27.0) < 27.0 * 1e-6, r["e0"]


def test_degenerate_suspect_flag(q):
    # near-degenerate: two identical dimers (t = -1) coupled by 1e-10, one up
    # electron: the lowest two one-body levels are -1 -+ 5e-11, which the
    # exhausted Krylov space resolves, so theta_1 - theta_0 ~ 1e-10 < 1e-8
    from oracle import dense
    t = np.zeros((4, 4))
    t[0, 1] = t[1, 0] = t[2, 3] = t[3, 2] = -1.0
    t[1, 2] = t[2, 1] = 1e-10
    U = np.full(4, 4.0)
    w = dense.ground_state(t, U, 1, 0)[2]
    assert w[1] - w[0] < 1e-8
    b = q.sector_basis(4, 1, 0)
    r = q.lanczos_gs((t, U), b)
    assert r["degenerate_suspect"], (r["e0"], r["theta1"])
    assert abs(r["e0"] - w[0]) < 1e-12
    # a non-degenerate ground state (the half-filled plaquette, gap > 0.1)
    m = synth.plaquette_2x2()
    wd = dense.ground_state(m.t, m.U, m.nup, m.ndn)[2]
    assert wd[1] - wd[0] > 0.1
    r2 = q.lanczos_gs(m, q.sector_basis(m.L, m.nup, m.ndn))
    assert r2["converged"] and not r2["degenerate_suspect"], r2["theta1"] - r2["e0"]


# ---------------------------------------------------------------- Green function and CPT

Z64 = synth.omega_grid()


# Chains are run past convergence: a truncated, unconverged chain without
# reorthogonalisation is chaotic in the rounding (a 1e-13 change of the ground
# state moves a 200-step G of the 7-orbital impurity by 4e-3), while converged
# chains of both sides reach the same Lehmann sum.
@pytest.mark.parametrize("m,steps", [(synth.plaquette_2x2(), 200), (synth.random_model(301, 6, 3, 2), 400),
                                     (synth.impurity_model(np.random.default_rng(18643), 3), 600)],
                         ids=lambda x: getattr(x, "name", str(x)))
def test_green_function(q, m, steps):
    print(f"green {m.name}", flush=True)
    b = q.sector_basis(m.L, m.nup, m.ndn)
    r = q.lanczos_gs(m, b)
    ro = oracle.lanczos_gs(m.t, m.U, m.nup, m.ndn, want_vector=True)
    orbs = list(range(min(m.L, 4)))
    g = q.green_cf(m, b, r["psi"], r["e0"], orbs, Z64, max_steps=steps)
    ch = oracle.green_cf(m.t, m.U, m.nup, m.ndn, ro["psi"], orbs, max_steps=steps)
    Go = cf.green_matrix(ch, len(orbs), Z64, ro["e0"])
    G = g["G"].cpu().numpy()
    err = np.abs(G - Go).max()
    print(f"  max |dG| = {err:.2e}")
    assert err <= 1e-4
    # b0^2 of every chain matches the oracle's
    p = 0
    for i in range(len(orbs)):
        for j in range(i, len(orbs)):
            for part in (0, 1):
                assert abs(g["coef"][p, part, 0] - ch[(i, j, part)][0]) < 1e-12
            p += 1


# Full reorthogonalisation (reorth = 2, a test device): truncated chains are
# the recurrence of exact arithmetic, so from the same start vectors the
# coefficients agree floor by floor and G agrees far below 1e-4, also before
# the Krylov space is exhausted.  Exhausted chains give the dense Lehmann sum.
# FP32 vectors: the storage rounding (relative 6e-8 per stored vector) is
# amplified by the truncated continued fraction (1.5e-4 measured on the
# 30-floor case); the error is printed and bounded at 2e-3.
@pytest.mark.parametrize("m,steps,exhaust", [(synth.random_model(43, 6, 3, 3), 30, False),
                                             (synth.random_model(301, 6, 3, 2), 40, False),
                                             (synth.random_model(42, 5, 2, 3), 120, True)],
                         ids=["rand6_30", "rand6b_40", "rand5_exhausted"])
@pytest.mark.parametrize("prec", ["fp64", "fp32v"])
def test_green_full_reorth(q, m, steps, exhaust, prec):
    torch = _torch()
    print(f"green full reorth {m.name} {steps} {prec}", flush=True)
    b = q.sector_basis(m.L, m.nup, m.ndn)
    ro = oracle.lanczos_gs(m.t, m.U, m.nup, m.ndn, want_vector=True, nthreads=1)
    psi = torch.from_numpy(ro["psi"]).to("cuda")
    orbs = list(range(m.L))
    g = q.green_cf(m, b, psi, ro["e0"], orbs, Z64, max_steps=steps, reorth=2, prec=prec)
    ch = oracle.green_cf(m.t, m.U, m.nup, m.ndn, ro["psi"], orbs, max_steps=steps,
                         full_reorth=True, nthreads=1)
    Go = cf.green_matrix(ch, len(orbs), Z64, ro["e0"])
    G = g["G"].cpu().numpy()
    err = np.abs(G - Go).max()
    print(f"  max |dG| = {err:.2e}")
    if exhaust:
        from oracle import dense
        Gd = dense.lehmann_green(m.t, m.U, m.nup, m.ndn, orbs, Z64, psi=ro["psi"], e0=ro["e0"])
        print(f"  max |dG| vs Lehmann = {np.abs(G - Gd).max():.2e}")
        assert np.abs(G - Gd).max() <= (1e-9 if prec == "fp64" else 2e-3)
    assert err <= (1e-9 if prec == "fp64" else 2e-3)
    M = g["coef"].shape[2] // 2
    p = 0
    worst = 0.0
    for i in range(len(orbs)):
        for j in range(i, len(orbs)):
            for part in (0, 1):
                b0, a, b2 = ch[(i, j, part)]
                co = g["coef"][p, part]
                assert g["len"][p, part] == len(a)
                assert abs(co[0] - b0) < (1e-12 if prec == "fp64" else 1e-6)
                # late floors are sensitive once Ritz values converge (G is
                # not): the first floors one by one
                k = min(len(a), 12 if prec == "fp64" else 4)
                worst = max(worst, np.abs(co[1:1 + k] - a[:k]).max() / max(1.0, np.abs(a).max()))
            p += 1
    print(f"  first floors: max |da| / max |a| = {worst:.2e}")
    assert worst <= (1e-9 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("prec", ["fp64", "fp32v"])
def test_green_long_rows(q, prec):
    """Continued fractions whose sectors have long rows (16 orbitals, ground
    state in (8, 1); the electron part (9, 1) and the hole part (7, 1) have
    rows of 11,440 strings): several chains per launch through the two-pass
    step, its dots and its deferred updates.  From the oracle's ground state,
    b0^2 of every chain to 1e-12 and the first 12 floors to 1e-9 (FP32
    vectors: 1e-6 and the first 4 floors to 1e-5)."""
    torch = _torch()
    m = synth.rect_cluster(4, 4, U=8.0, mu=4.0, nup=8, ndn=1, name="4x4r")
    print(f"green long rows {m.name} {prec}", flush=True)
    b = q.sector_basis(m.L, m.nup, m.ndn)
    ro = oracle.lanczos_gs(m.t, m.U, m.nup, m.ndn, want_vector=True)
    psi = torch.from_numpy(ro["psi"]).to("cuda")
    orbs = [0, 5, 10, 15]
    g = q.green_cf(m, b, psi, ro["e0"], orbs, Z64, max_steps=12, prec=prec,
                   reorth=1 if prec == "fp32v" else 0)
    ch = oracle.green_cf(m.t, m.U, m.nup, m.ndn, ro["psi"], orbs, max_steps=12)
    p = 0
    worst = worst_b0 = 0.0
    for i in range(len(orbs)):
        for j in range(i, len(orbs)):
            for part in (0, 1):
                b0, a, b2 = ch[(i, j, part)]
                co = g["coef"][p, part]
                worst_b0 = max(worst_b0, abs(co[0] - b0))
                k = min(len(a), 12 if prec == "fp64" else 4)
                worst = max(worst, np.abs(co[1:1 + k] - a[:k]).max() / max(1.0, np.abs(a).max()))
            p += 1
    print(f"  b0^2 {worst_b0:.2e}; first floors: max |da| / max |a| = {worst:.2e}")
    assert worst_b0 <= (1e-12 if prec == "fp64" else 1e-6)
    assert worst <= (1e-9 if prec == "fp64" else 1e-5)


def test_cpt_2x2(q):
    torch = _torch()
    m = synth.plaquette_2x2()
    ro = oracle.lanczos_gs(m.t, m.U, 2, 2, want_vector=True)
    ch = oracle.green_cf(m.t, m.U, 2, 2, ro["psi"], [0, 1, 2, 3])
    Go = cf.green_matrix(ch, 4, Z64, ro["e0"])
    R, E, bonds = synth.cpt_square_lattice_2x2()
    ks = synth.k_grid_2d(16)
    gp = q.cpt_gk(torch.from_numpy(Go).to("cuda"), R, E, bonds, ks).cpu().numpy()
    gpo = cf.cpt_periodized(Go, R, E, bonds, ks)
    assert np.abs(gp - gpo).max() <= 1e-10


def test_hv_plan_matches_hv(q):
    torch = _torch()
    # short rows (fused product kernel and the one-row-per-block kernel) and
    # long rows (the two-pass path, uniform and per-bond t)
    for m in (synth.cluster_3x4(), synth.random_model(102, 11, 3, 6),
              synth.rect_cluster(4, 4, U=8.0, mu=4.0, nup=8, ndn=1, name="4x4r"),
              synth.rect_cluster(5, 3, tp=0.3, U=5.0, mu=2.5, nup=7, ndn=2, name="5x3r")):
        b = q.sector_basis(m.L, m.nup, m.ndn)
        for dt, prec in ((torch.float64, "fp64"), (torch.float32, "fp32v")):
            v = (torch.rand(2 * b.dim, dtype=torch.float64, device="cuda") * 2 - 1).to(dt)
            plan = q.HvPlan(m, b, prec)
            w2 = torch.empty_like(v)
            plan(v, w2, nvec=2)
            for k in range(2):
                w1 = q.hv(m, b, v[k * b.dim:(k + 1) * b.dim].contiguous())
                assert torch.equal(w1, w2[k * b.dim:(k + 1) * b.dim])
            with pytest.raises(q.QcmError):
                plan(v, v, nvec=2)
            plan.close()


# ---------------------------------------------------------------- band Lanczos
#
# A band Lanczos G on a truncated basis depends on its start states with a
# large condition number (the Krylov space holds H^k of them): in the oracle
# alone, a perturbation of psi of norm 1e-15 moves G(z) on rand504_L7 by 6e-10
# at R = 24 and by 1.4e-7 at R = 30.  So the recurrence is compared from the
# same start states (the oracle's psi and E0 on both sides), at basis sizes
# where that amplification stays below 1e-9; the whole path from the GPU's own
# ground state is compared through the spectral moments Q Lambda^k Q^T, which
# depend smoothly on psi.

BAND_CASES = [(synth.plaquette_2x2(), [0, 1, 2, 3], 24),
              (synth.chain(8, U=4.0, mu=2.0, nup=4, ndn=4), [0, 1, 2, 3], 24),
              (synth.impurity_model(np.random.default_rng(18643), 3), [0, 1, 2, 3], 40),
              (synth.random_model(504, 7, 3, 4), [0, 3, 6], 24)]
BAND_IDS = ["2x2", "chain8", "imp7", "rand7"]


def _moments(lam, Q, k):
    """Q diag(Lambda^k) Q^T = B^T H^k B for the start block B of one part."""
    return (Q * lam ** k) @ Q.T


@pytest.mark.parametrize("m,orbs,R", BAND_CASES, ids=BAND_IDS)
def test_band_lanczos(q, m, orbs, R):
    """The GPU band Lanczos against the oracle's (the paper's recurrence, same
    start states, same basis size, short enough that orthogonality holds): G
    to 1e-8, Lambda to 1e-8, the same R; Q Q^T = 1 over both parts to 1e-12."""
    from oracle import band
    torch = _torch()
    print(f"band {m.name} R={R}", flush=True)
    b = q.sector_basis(m.L, m.nup, m.ndn)
    ro = oracle.lanczos_gs(m.t, m.U, m.nup, m.ndn, want_vector=True)
    psi = torch.from_numpy(ro["psi"]).to("cuda")
    g = q.green_band(m, b, psi, ro["e0"], orbs, Z64, max_basis=R)
    Go, parts = band.green_band(m.t, m.U, m.nup, m.ndn, ro["psi"], orbs, ro["e0"], Z64, max_basis=R)
    err = np.abs(g["G"].cpu().numpy() - Go).max()
    print(f"  R {list(g['R'])}, max |dG| {err:.2e}")
    assert err <= 1e-8
    for k in range(2):
        assert g["R"][k] == parts[k][0].shape[0]
        assert np.abs(np.sort(g["lam"][k]) - np.sort(parts[k][0])).max() <= 1e-8
    Q = np.concatenate(g["Q"], axis=1)
    assert np.abs(Q @ Q.T - np.eye(len(orbs))).max() <= 1e-12


@pytest.mark.parametrize("m,orbs,R", BAND_CASES, ids=BAND_IDS)
def test_band_lanczos_from_gpu_ground_state(q, m, orbs, R):
    """The whole path on the GPU (its own ground state, then band Lanczos):
    for each part, Q Lambda^k Q^T = B^T H^k B for k = 0..3 (exact for a band
    Lanczos run of at least two blocks), against the oracle's, relative 1e-9
    of the largest entry."""
    from oracle import band
    print(f"band moments {m.name} R={R}", flush=True)
    b = q.sector_basis(m.L, m.nup, m.ndn)
    r = q.lanczos_gs(m, b)
    ro = oracle.lanczos_gs(m.t, m.U, m.nup, m.ndn, want_vector=True)
    g = q.green_band(m, b, r["psi"], r["e0"], orbs, Z64, max_basis=R)
    _, parts = band.green_band(m.t, m.U, m.nup, m.ndn, ro["psi"], orbs, ro["e0"], Z64, max_basis=R)
    worst = 0.0
    for part in range(2):
        for k in range(4):
            Mg = _moments(g["lam"][part], g["Q"][part], k)
            Mo = _moments(parts[part][0], parts[part][1], k)
            worst = max(worst, np.abs(Mg - Mo).max() / max(1.0, np.abs(Mo).max()))
    print(f"  moments 0..3: max relative difference {worst:.2e}")
    assert worst <= 1e-9


@pytest.mark.parametrize("m,orbs", [(synth.random_model(501, 6, 3, 2), [0, 2, 5]),
                                    (synth.chain(8, U=4.0, mu=2.0, nup=4, ndn=4), [0, 1, 2, 3]),
                                    (synth.impurity_model(np.random.default_rng(18643), 3), [0, 1, 2, 3]),
                                    (synth.chain(10, U=4.0, mu=2.0, nup=5, ndn=5), list(range(10)))],
                         ids=["rand6", "chain8", "imp7", "chain10"])
def test_band_lanczos_stopping_rule(q, m, orbs):
    """The paper's stopping rule (lowest eigenvalue of T converged to 1e-10,
    tested once per block) on the GPU and in the oracle, from the same start
    states: the same basis size R per part, the same lowest Ritz value
    (relative 1e-10), the moments B^T H^k B for k = 0..3 (relative 1e-9) and
    Q Q^T = 1 (1e-12).  The converged G is printed, not compared: past the
    point where orthogonality leaks it depends on rounding."""
    from oracle import band
    torch = _torch()
    print(f"band stop {m.name} p={len(orbs)}", flush=True)
    b = q.sector_basis(m.L, m.nup, m.ndn)
    ro = oracle.lanczos_gs(m.t, m.U, m.nup, m.ndn, want_vector=True)
    psi = torch.from_numpy(ro["psi"]).to("cuda")
    g = q.green_band(m, b, psi, ro["e0"], orbs, Z64, max_basis=1000, etol=1e-10)
    Go, parts = band.green_band(m.t, m.U, m.nup, m.ndn, ro["psi"], orbs, ro["e0"], Z64,
                                max_basis=1000, etol=1e-10)
    err = np.abs(g["G"].cpu().numpy() - Go).max()
    print(f"  R {list(g['R'])} (oracle {[x[0].shape[0] for x in parts]}), max |dG| {err:.2e}")
    worst = 0.0
    for part in range(2):
        assert g["R"][part] == parts[part][0].shape[0]
        lg, lo = g["lam"][part].min(), parts[part][0].min()
        assert abs(lg - lo) <= 1e-10 * max(1.0, abs(lo))
        for k in range(4):
            Mg = _moments(g["lam"][part], g["Q"][part], k)
            Mo = _moments(parts[part][0], parts[part][1], k)
            worst = max(worst, np.abs(Mg - Mo).max() / max(1.0, np.abs(Mo).max()))
    print(f"  moments 0..3: max relative difference {worst:.2e}")
    assert worst <= 1e-9
    Q = np.concatenate(g["Q"], axis=1)
    assert np.abs(Q @ Q.T - np.eye(len(orbs))).max() <= 1e-12


def _deep_model():
    """Orbital 0 far below the others: always occupied, so c+_0 |Omega> = 0
    and the band recurrence must deflate that start state at once."""
    m = synth.random_model(502, 6, 3, 3)
    t = m.t.copy()
    t[0, 0] = -40.0
    return synth.Model("deep6", t, m.U, 3, 3)


@pytest.mark.parametrize("m,orbs", [(synth.random_model(505, 6, 0, 3), [0, 2, 4]),
                                    (synth.random_model(506, 6, 6, 2), [1, 3, 5]),
                                    (_deep_model(), [0, 2, 4])],
                         ids=["empty_up", "full_up", "vanishing_start"])
def test_band_lanczos_edge_sectors(q, m, orbs):
    """Band Lanczos where a part does not exist (N_up = 0: no hole part;
    N_up = L: no electron part) or a start state vanishes (deflated at once):
    the same R per part as the oracle, G to 1e-8 from the same start states,
    and Q Q^T = 1 over what exists (the anticommutator needs both parts only
    where both exist)."""
    from oracle import band
    torch = _torch()
    print(f"band edge {m.name} ({m.nup},{m.ndn})", flush=True)
    b = q.sector_basis(m.L, m.nup, m.ndn)
    ro = oracle.lanczos_gs(m.t, m.U, m.nup, m.ndn, want_vector=True)
    psi = torch.from_numpy(ro["psi"]).to("cuda")
    g = q.green_band(m, b, psi, ro["e0"], orbs, Z64, max_basis=12)
    Go, parts = band.green_band(m.t, m.U, m.nup, m.ndn, ro["psi"], orbs, ro["e0"], Z64,
                                max_basis=12)
    err = np.abs(g["G"].cpu().numpy() - Go).max()
    print(f"  R {list(g['R'])} (oracle {[x[0].shape[0] for x in parts]}), max |dG| {err:.2e}")
    for k in range(2):
        assert g["R"][k] == parts[k][0].shape[0]
    if m.nup == 0:
        assert g["R"][1] == 0
    if m.nup == m.L:
        assert g["R"][0] == 0
    assert err <= 1e-8
    Q = np.concatenate(g["Q"], axis=1)
    assert np.abs(Q @ Q.T - np.eye(len(orbs))).max() <= 1e-12


def test_band_lanczos_many_orbitals(q):
    """16 start states and up to 800 basis vectors per part, so that the
    start-state projections (p R doubles) exceed the 96 KB the eigen-solver
    of T keeps in LDS and its global-memory path runs: for each part the
    moments Q Lambda^k Q^T against B^T H^k B formed directly from the
    oracle's start states and products (k <= 3, relative 1e-9), and
    Q Q^T = 1 over both parts (1e-12)."""
    torch = _torch()
    m = synth.random_model(507, 16, 2, 1)
    orbs = list(range(16))
    print(f"band many orbitals {m.name} p={len(orbs)}", flush=True)
    b = q.sector_basis(m.L, m.nup, m.ndn)
    ro = oracle.lanczos_gs(m.t, m.U, m.nup, m.ndn, want_vector=True)
    psi = torch.from_numpy(ro["psi"]).to("cuda")
    g = q.green_band(m, b, psi, ro["e0"], orbs, Z64, max_basis=800)
    print(f"  R {list(g['R'])}")
    assert max(g["R"]) * len(orbs) * 8 > 96 * 1024
    worst = 0.0
    for part in range(2):
        nup2 = m.nup + 1 if part == 0 else m.nup - 1
        B = np.stack([oracle.apply_op(m.L, m.nup, m.ndn, ro["psi"], part, mu) for mu in orbs],
                     axis=1)
        X = B.copy()
        for k in range(4):
            Mo = B.T @ X
            Mg = _moments(g["lam"][part], g["Q"][part], k)
            worst = max(worst, np.abs(Mg - Mo).max() / max(1.0, np.abs(Mo).max()))
            X = np.stack([oracle.hv(m.t, m.U, nup2, m.ndn, X[:, i]) for i in range(len(orbs))],
                         axis=1)
    print(f"  moments 0..3: max relative difference {worst:.2e}")
    assert worst <= 1e-9
    Q = np.concatenate(g["Q"], axis=1)
    assert np.abs(Q @ Q.T - np.eye(len(orbs))).max() <= 1e-12


@pytest.mark.parametrize("R", [1, 2, 3, 7])
def test_band_lanczos_one_orbital_short(q, R):
    """One start state and 1, 2, 3 or 7 basis vectors per part: T of size 1
    (no reduction, no QR step), 2 (QR steps only) and larger, against the
    oracle's run from the same start state: R, Lambda and G to 1e-10."""
    from oracle import band
    torch = _torch()
    m = synth.random_model(508, 6, 3, 3)
    orbs = [2]
    print(f"band one orbital R={R}", flush=True)
    b = q.sector_basis(m.L, m.nup, m.ndn)
    ro = oracle.lanczos_gs(m.t, m.U, m.nup, m.ndn, want_vector=True)
    psi = torch.from_numpy(ro["psi"]).to("cuda")
    g = q.green_band(m, b, psi, ro["e0"], orbs, Z64, max_basis=R)
    Go, parts = band.green_band(m.t, m.U, m.nup, m.ndn, ro["psi"], orbs, ro["e0"], Z64,
                                max_basis=R)
    err = np.abs(g["G"].cpu().numpy() - Go).max()
    print(f"  R {list(g['R'])}, max |dG| {err:.2e}")
    assert err <= 1e-10
    for k in range(2):
        assert g["R"][k] == parts[k][0].shape[0] == R
        assert np.abs(np.sort(g["lam"][k]) - np.sort(parts[k][0])).max() <= 1e-10


def test_band_lanczos_one_orbital_stopping_rule(q):
    """One start state with the paper's stopping rule (tested after every
    basis vector, from T of size 1 on): the same R per part as the oracle and
    the same lowest Ritz value (relative 1e-10)."""
    from oracle import band
    torch = _torch()
    m = synth.random_model(508, 6, 3, 3)
    orbs = [2]
    b = q.sector_basis(m.L, m.nup, m.ndn)
    ro = oracle.lanczos_gs(m.t, m.U, m.nup, m.ndn, want_vector=True)
    psi = torch.from_numpy(ro["psi"]).to("cuda")
    g = q.green_band(m, b, psi, ro["e0"], orbs, Z64, max_basis=200, etol=1e-10)
    _, parts = band.green_band(m.t, m.U, m.nup, m.ndn, ro["psi"], orbs, ro["e0"], Z64,
                               max_basis=200, etol=1e-10)
    print(f"band one orbital stop: R {list(g['R'])} (oracle {[x[0].shape[0] for x in parts]})")
    for k in range(2):
        assert g["R"][k] == parts[k][0].shape[0]
        lg, lo = g["lam"][k].min(), parts[k][0].min()
        assert abs(lg - lo) <= 1e-10 * max(1.0, abs(lo))


def test_band_lanczos_fp32v_errors_reported(q):
    """FP32 vectors (FP64 sums and coefficients): against the FP64 run from
    the same start states, the lowest Ritz value of each part and the
    moments B^T H^k B (k <= 3) to relative 1e-5, G reported."""
    torch = _torch()
    m = synth.chain(10, U=4.0, mu=2.0, nup=5, ndn=5)
    orbs = list(range(10))
    b = q.sector_basis(m.L, m.nup, m.ndn)
    ro = oracle.lanczos_gs(m.t, m.U, m.nup, m.ndn, want_vector=True)
    psi = torch.from_numpy(ro["psi"]).to("cuda")
    g64 = q.green_band(m, b, psi, ro["e0"], orbs, Z64, max_basis=60)
    g32 = q.green_band(m, b, psi, ro["e0"], orbs, Z64, max_basis=60, prec="fp32v")
    dG = np.abs(g64["G"].cpu().numpy() - g32["G"].cpu().numpy()).max()
    worst = 0.0
    for part in range(2):
        assert g32["R"][part] == g64["R"][part]
        l64, l32 = g64["lam"][part].min(), g32["lam"][part].min()
        assert abs(l64 - l32) <= 1e-5 * abs(l64)
        for k in range(4):
            M64 = _moments(g64["lam"][part], g64["Q"][part], k)
            M32 = _moments(g32["lam"][part], g32["Q"][part], k)
            worst = max(worst, np.abs(M64 - M32).max() / max(1.0, np.abs(M64).max()))
    print(f"  band FP32V vs FP64: moments {worst:.2e}, max |dG| {dG:.2e}")
    assert worst <= 1e-5
    Q = np.concatenate(g32["Q"], axis=1)
    assert np.abs(Q @ Q.T - np.eye(len(orbs))).max() <= 1e-6
