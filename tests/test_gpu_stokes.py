"""GPU parity of the Stokes path through the C ABI against the CPU oracle.

Inputs are seeded (paper_2303_10233_amd.workloads); expected values come from
oracle/ only.  Tolerances: FP64 operator and preconditioner applies agree to
rounding (1e-12 relative); FP32 (mixed) preconditioner applies to 1e-5
relative (single-precision rounding through the multigrid levels and 20
Chebyshev steps); FP64 solves at rtol 1e-12 to 1e-8 relative in the
canonicalised full vector (the FP64 bar of 1e-8).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle.assemble import Mesh, System, lid_dirichlet  # noqa: E402
from oracle.direct import direct_solve, canonicalize, rel_err  # noqa: E402
from oracle import precond as opc  # noqa: E402
from oracle.krylov import minres  # noqa: E402
from paper_2303_10233_amd import eth  # noqa: E402
from paper_2303_10233_amd.workloads import gaussian_bumps, uniform_vector  # noqa: E402

DEV = "cuda:0"


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    eth.load_library()


@pytest.mark.parametrize("n", [2, 3, 5, 16, 33, 64])
def test_apply_operator_matches_oracle(n):
    print(f"[apply] n={n}", flush=True)
    m = Mesh(n)
    s = System(m, nu=0.7)
    P = eth.Problem(n, nu=0.7, velocity=eth.VEL_EXACT if n <= 32 else eth.VEL_GMG,
                    mq=eth.MQ_DIAG, max_batch=3)
    xs = [uniform_vector(m.N, 100 + n + k) for k in range(3)]
    # batch of three with a padded stride
    ld = m.N + 17
    X = torch.zeros((3, ld), dtype=torch.float64, device=DEV)
    for k in range(3):
        X[k, : m.N] = _t(xs[k])
    Y = P.apply_operator(X)
    Yn = _np(Y)
    for k in range(3):
        ref = s.apply_full(xs[k])
        assert rel_err(Yn[k, : m.N], ref) < 1e-13
    # single vector
    y1 = _np(P.apply_operator(_t(xs[0])))
    assert rel_err(y1, s.apply_full(xs[0])) < 1e-13


@pytest.mark.parametrize("n", [16, 33, 64])
def test_apply_with_xcd_band_order_matches_oracle(n, monkeypatch):
    """Large grids of the apply renumber their tiles by XCD band; forced on
    small grids here, the operator still equals the oracle's and its fused
    dot is unchanged up to the summation order."""
    monkeypatch.setenv("ETH_DEBUG_XCD_REMAP_MIN", "1")
    m = Mesh(n)
    s = System(m, nu=0.7)
    P = eth.Problem(n, nu=0.7)
    x = uniform_vector(m.N, 5 + n)
    y = _np(P.apply_operator(_t(x)))
    assert rel_err(y, s.apply_full(x)) < 1e-13
    monkeypatch.setenv("ETH_DEBUG_XCD_REMAP_MIN", "1000000000")
    y2 = _np(P.apply_operator(_t(x)))
    assert np.array_equal(y, y2)


@pytest.mark.parametrize("prec", [eth.FP64, eth.MIXED])
def test_vcycle_with_xcd_band_order_is_bitwise_the_same(prec, monkeypatch):
    """The smoother and restriction renumber large grids by XCD band; forced
    on at n = 96 every tile is still computed once, so the preconditioner's
    output is bit for bit the plain-order one."""
    n = 96
    m = Mesh(n)
    r = uniform_vector(m.N, 21)
    r[: 2 * m.nv][System(m).vel_bnd] = 0.0
    P = eth.Problem(n, precision=prec, velocity=eth.VEL_GMG, mq=eth.MQ_DIAG)
    z0 = _np(P.apply_preconditioner(_t(r)))
    monkeypatch.setenv("ETH_DEBUG_XCD_REMAP_MIN", "1")
    z1 = _np(P.apply_preconditioner(_t(r)))
    assert np.array_equal(z0, z1)


def test_operator_symmetric_and_frame_null_vector():
    n = 24
    m = Mesh(n)
    P = eth.Problem(n, mq=eth.MQ_DIAG)
    x = _t(uniform_vector(m.N, 1))
    y = _t(uniform_vector(m.N, 2))
    Ax, Ay = P.apply_operator(x), P.apply_operator(y)
    # boundary velocity entries are ignored: compare on the interior layout
    s = System(m)
    xi, yi = s.to_interior(_np(x)), s.to_interior(_np(y))
    a = s.to_interior(_np(Ay)) @ xi
    b = s.to_interior(_np(Ax)) @ yi
    assert abs(a - b) <= 1e-13 * (abs(a) + abs(b))
    k = np.zeros(m.N)
    k[2 * m.nv: 2 * m.nv + m.nk] = 1.0
    k[2 * m.nv + m.nk:] = -1.0
    Ak = _np(P.apply_operator(_t(k)))
    assert np.abs(Ak).max() < 1e-14


@pytest.mark.parametrize("n", [4, 33])
@pytest.mark.parametrize("corner_mode", [0, 1])
def test_assemble_rhs_matches_oracle(n, corner_mode):
    print(f"[rhs] n={n} corner_mode={corner_mode}", flush=True)
    m = Mesh(n)
    nu = 0.3
    s = System(m, nu=nu)
    P = eth.Problem(n, nu=nu, lid_u=1.5, corner_mode=corner_mode, mq=eth.MQ_DIAG,
                    max_batch=2)
    f = gaussian_bumps(n, 1000)
    b = _np(P.assemble_rhs(_t(f)))
    ref = s.rhs(f, lid_dirichlet(m, 1.5, corner_mode))
    assert rel_err(b, ref) < 1e-13
    b0 = _np(P.assemble_rhs(None))
    assert rel_err(b0, s.rhs(None, lid_dirichlet(m, 1.5, corner_mode))) < 1e-13
    # batched forcing
    F = torch.stack([_t(gaussian_bumps(n, 1001)), _t(gaussian_bumps(n, 1002))])
    B = _np(P.assemble_rhs(F, batch=2))
    for k in range(2):
        assert rel_err(B[k], s.rhs(gaussian_bumps(n, 1001 + k), lid_dirichlet(m, 1.5, corner_mode))) < 1e-13


def _mq_lo(n):
    return min(0.01, 0.4 / n)


def _oracle_prec(s, velocity, mq, lambdas=None, mq_lo=None):
    gmg_kw = dict(lambdas=lambdas) if lambdas is not None else None
    lo = _mq_lo(s.mesh.n) if mq_lo is None else mq_lo
    return opc.StokesBlockDiag(s, velocity, mq, mq_lo=lo, mq_steps=20, gmg_kw=gmg_kw)


def _oracle_lambdas(n):
    g = opc.GMG(Mesh(n), opc.laplacian)
    return g.lam


@pytest.mark.parametrize("n,velocity,mq,prec,tol", [
    (8, "exact", "diag", eth.FP64, 1e-12),
    (16, "exact", "diag", eth.FP64, 1e-12),
    (16, "gmg", "cheb_sgs", eth.FP64, 1e-11),
    (48, "gmg", "cheb_sgs", eth.FP64, 1e-11),
    (64, "gmg", "diag", eth.FP64, 1e-11),
    (64, "gmg", "cheb_sgs", eth.MIXED, 2e-5),
])
def test_preconditioner_matches_oracle(n, velocity, mq, prec, tol):
    print(f"[precond] n={n} {velocity} {mq} prec={prec}", flush=True)
    m = Mesh(n)
    nu = 0.5
    s = System(m, nu=nu)
    lam = _oracle_lambdas(n) if velocity == "gmg" else None
    P = eth.Problem(n, nu=nu, velocity=eth.VEL_GMG if velocity == "gmg" else eth.VEL_EXACT,
                    mq=eth.MQ_DIAG if mq == "diag" else eth.MQ_CHEB_SGS, precision=prec,
                    gmg_lambda=lam, mq_cheb=(_mq_lo(n), 1.0))
    r = uniform_vector(m.N, 7 + n)
    r[: 2 * m.nv][s.vel_bnd] = 0.0
    z = _np(P.apply_preconditioner(_t(r)))
    Pref = _oracle_prec(s, velocity, mq, lambdas=lam)
    zref = s.to_full(Pref(s.to_interior(r)))
    o = 2 * m.nv
    assert rel_err(z[:o], zref[:o]) < tol
    assert rel_err(z[o:], zref[o:]) < tol
    assert np.abs(z[:o][s.vel_bnd]).max() == 0.0


@pytest.mark.parametrize("n,prec,tol", [(128, eth.FP64, 1e-12), (48, eth.FP64, 1e-12),
                                        (256, eth.MIXED, 1e-5), (96, eth.MIXED, 1e-5)])
def test_fused_coarse_vcycle_equals_per_level_launches(n, prec, tol, monkeypatch):
    """The coarse end of the V-cycle in one launch (levels <= 32^2 in LDS)
    against one launch per level step: identical node arithmetic, so only the
    coarsest dense product (summation order) differs."""
    print(f"[fused vcycle] n={n} prec={prec}", flush=True)
    m = Mesh(n)
    r = uniform_vector(m.N, 11 + n)
    r[: 2 * m.nv][System(m).vel_bnd] = 0.0
    P = eth.Problem(n, precision=prec, velocity=eth.VEL_GMG, mq=eth.MQ_DIAG)
    z_fused = _np(P.apply_preconditioner(_t(r)))
    monkeypatch.setenv("ETH_DEBUG_UNFUSED_VCYCLE", "1")
    Q = eth.Problem(n, precision=prec, velocity=eth.VEL_GMG, mq=eth.MQ_DIAG)
    z_ref = _np(Q.apply_preconditioner(_t(r)))
    o = 2 * m.nv
    assert rel_err(z_fused[:o], z_ref[:o]) < tol
    assert np.array_equal(z_fused[o:], z_ref[o:])


@pytest.mark.parametrize("n,prec", [(16, eth.FP64), (64, eth.FP64), (96, eth.FP64), (256, eth.FP64),
                                    (40, eth.MIXED), (128, eth.MIXED), (256, eth.MIXED)])
def test_fused_smoothing_launches_equal_per_step_launches(n, prec, monkeypatch):
    """V(2,2) with the second pre-smoothing step inside the restriction's
    launch and the correction plus both post-smoothing steps in one launch
    per level, against one launch per step: the same node expressions in the
    same order.  In FP32 (the mixed-precision preconditioner) the two agree
    bit for bit, preconditioner and whole graph-replayed solve; in FP64 the
    compiler contracts a few multiply-adds differently in the two code
    shapes, which leaves differences at the rounding level (measured up to
    7e-14 absolute at 256^2)."""
    print(f"[fused smoothing] n={n} prec={prec}", flush=True)
    m = Mesh(n)
    r = uniform_vector(m.N, 21 + n)
    r[: 2 * m.nv][System(m).vel_bnd] = 0.0
    monkeypatch.setenv("ETH_DEBUG_UNFUSED_SMOOTH", "0")
    P = eth.Problem(n, precision=prec, velocity=eth.VEL_GMG, mq=eth.MQ_DIAG)
    z_fused = _np(P.apply_preconditioner(_t(r)))
    b = P.assemble_rhs()
    # FP64: solved far enough that a one-iteration difference in where the
    # two stop does not show in the comparison
    rtol = 1e-8 if prec == eth.MIXED else 1e-12
    x_fused, i_fused = P.solve(b, rtol=rtol, maxit=2000, use_graph=True)
    x_fused = _np(x_fused)
    monkeypatch.setenv("ETH_DEBUG_UNFUSED_SMOOTH", "1")
    Q = eth.Problem(n, precision=prec, velocity=eth.VEL_GMG, mq=eth.MQ_DIAG)
    z_ref = _np(Q.apply_preconditioner(_t(r)))
    x_ref, i_ref = Q.solve(Q.assemble_rhs(), rtol=rtol, maxit=2000, use_graph=True)
    o = 2 * m.nv
    print(f"  max |dz| = {np.abs(z_fused - z_ref).max():.3e}", flush=True)
    print(f"  iterations {i_fused[0]['iterations']} / {i_ref[0]['iterations']}, status "
          f"{i_fused[0]['status']} / {i_ref[0]['status']}", flush=True)
    if prec == eth.MIXED:
        assert np.array_equal(z_fused[:o], z_ref[:o])
        assert i_fused[0]["iterations"] == i_ref[0]["iterations"]
        assert np.array_equal(x_fused, _np(x_ref))
    else:
        assert rel_err(z_fused[:o], z_ref[:o]) < 1e-13
        if n <= 128:   # the diagonal pressure block needs more than maxit beyond
            assert i_fused[0]["status"] == 0 and i_ref[0]["status"] == 0
            assert abs(i_fused[0]["iterations"] - i_ref[0]["iterations"]) <= 2
            assert rel_err(x_fused, _np(x_ref)) < 1e-9


@pytest.mark.parametrize("n,prec", [(8, eth.FP64), (16, eth.FP64), (66, eth.FP64), (12, eth.MIXED),
                                    (64, eth.MIXED), (132, eth.MIXED)])
def test_fused_cheb_sgs_step_equals_per_colour_passes(n, prec, monkeypatch):
    """The temporally blocked Chebyshev-SGS kernel (nine colour passes in LDS
    per launch, the input projection folded into the first) reproduces the
    one-launch-per-colour sweep bit for bit, for every tile side: n a multiple
    of the side (the last tiles of each row and column also own node n), n
    below it (one tile), and ragged edge tiles."""
    m = Mesh(n)
    r = uniform_vector(m.N, 3 + n)
    r[: 2 * m.nv][System(m).vel_bnd] = 0.0
    o = 2 * m.nv
    tiles = [8, 16, 24, 32] + ([64] if prec == eth.MIXED else [])
    z_fused = {}
    for tile in tiles:
        print(f"[fused mq] n={n} prec={prec} tile={tile}", flush=True)
        P = eth.Problem(n, precision=prec, velocity=eth.VEL_GMG, mq_tile=tile)
        assert P.mq_tile() == (tile, tile)
        z_fused[tile] = _np(P.apply_preconditioner(_t(r)))
    A = eth.Problem(n, precision=prec, velocity=eth.VEL_GMG)
    assert A.mq_tile()[0] in tiles
    monkeypatch.setenv("ETH_DEBUG_UNFUSED_MQ", "1")
    Q = eth.Problem(n, precision=prec, velocity=eth.VEL_GMG)
    z_plain = _np(Q.apply_preconditioner(_t(r)))
    for tile in tiles:
        assert np.array_equal(z_fused[tile][o:], z_plain[o:]), tile
    if prec == eth.MIXED:
        # two Chebyshev steps per launch (halo 20), also with an odd step count
        for steps in (20, 7):
            monkeypatch.setenv("ETH_DEBUG_UNFUSED_MQ", "1")
            Q2 = eth.Problem(n, precision=prec, velocity=eth.VEL_GMG, mq_steps=steps)   # per colour
            zq = _np(Q2.apply_preconditioner(_t(r)))
            monkeypatch.delenv("ETH_DEBUG_UNFUSED_MQ")
            for tile in (16, 24):
                print(f"[fused mq] n={n} two steps per launch, tile {tile}, mq_steps={steps}", flush=True)
                A2 = eth.Problem(n, precision=prec, velocity=eth.VEL_GMG, mq_tile=tile, mq_fuse_steps=2,
                                 mq_steps=steps)
                assert A2.mq_variant()[:2] == (tile, 2)
                z2 = _np(A2.apply_preconditioner(_t(r)))
                assert np.array_equal(z2[o:], zq[o:]), (tile, steps)


def test_two_steps_per_launch_solve_equals_one():
    """MINRES with the two-step fused kernel (the last launch writing straight
    to the FP64 vector) gives the one-step result bit for bit."""
    n = 64
    P1 = eth.Problem(n, precision=eth.MIXED, mq_tile=16, mq_fuse_steps=1)
    P2 = eth.Problem(n, precision=eth.MIXED, mq_tile=16, mq_fuse_steps=2)
    b = P1.assemble_rhs()
    x1, i1 = P1.solve(b, rtol=1e-8, maxit=500, use_graph=True)
    x2, i2 = P2.solve(b, rtol=1e-8, maxit=500, use_graph=True)
    assert i1[0]["iterations"] == i2[0]["iterations"]
    assert torch.equal(x1, x2)
    with pytest.raises(Exception):
        eth.Problem(16, precision=eth.FP64, mq_fuse_steps=2)
    with pytest.raises(Exception):
        eth.Problem(16, precision=eth.MIXED, mq_tile=32, mq_fuse_steps=2)


@pytest.mark.parametrize("prec", [eth.FP64, eth.MIXED])
def test_concurrent_blocks_equal_serial_preconditioner(prec, monkeypatch):
    """The pressure block runs on a second stream beside the V-cycle (a
    parallel branch of the captured graph): preconditioner and graph-replayed
    solves are bit for bit those of the serial order."""
    n = 64
    print(f"[concurrent precond] n={n} prec={prec}", flush=True)
    m = Mesh(n)
    r = uniform_vector(m.N, 17)
    r[: 2 * m.nv][System(m).vel_bnd] = 0.0
    P = eth.Problem(n, precision=prec, velocity=eth.VEL_GMG, mq_tile=16)
    z1 = _np(P.apply_preconditioner(_t(r)))
    b = P.assemble_rhs()
    x1, i1 = P.solve(b, rtol=1e-10, maxit=500, use_graph=True)
    monkeypatch.setenv("ETH_DEBUG_SERIAL_PRECOND", "1")
    Q = eth.Problem(n, precision=prec, velocity=eth.VEL_GMG, mq_tile=16)
    z2 = _np(Q.apply_preconditioner(_t(r)))
    x2, i2 = Q.solve(Q.assemble_rhs(), rtol=1e-10, maxit=500, use_graph=True)
    assert np.array_equal(z1, z2)
    assert i1[0]["iterations"] == i2[0]["iterations"]
    assert torch.equal(x1, x2)


@pytest.mark.parametrize("prec", [eth.FP64, eth.MIXED])
def test_timed_variant_solve_equals_forced_variant(prec):
    """The fused pressure-mass variant that set-up picks by timing (on whole
    applications of the concurrent preconditioner) is one of the offered
    ones, and a problem built with that variant forced solves bit for bit
    the same."""
    n = 64
    A = eth.Problem(n, precision=prec)
    tile, steps, tile_hi, steps_hi = A.mq_variant()
    assert (tile, steps) in [(8, 1), (16, 1), (24, 1), (32, 1), (16, 2), (24, 2), (64, 1)]
    assert steps == 1 or (prec == eth.MIXED and tile in (16, 24))
    F = eth.Problem(n, precision=prec, mq_tile=tile, mq_fuse_steps=steps)
    b = A.assemble_rhs()
    xa, ia = A.solve(b, rtol=1e-8, maxit=500, use_graph=True)
    xf, jf = F.solve(b, rtol=1e-8, maxit=500, use_graph=True)
    assert ia[0]["iterations"] == jf[0]["iterations"]
    assert torch.equal(xa, xf)


def test_mq_tile_rejects_unsupported_sides():
    with pytest.raises(Exception):
        eth.Problem(16, mq_tile=20)
    with pytest.raises(Exception):
        eth.Problem(16, precision=eth.MIXED, mq_tile=64, mq_fuse_steps=2)
    with pytest.raises(Exception):
        eth.Problem(16, precision=eth.FP64, mq_tile=64)


def test_gpu_lanczos_lambda_close_to_exact():
    """The set-up estimate of lambda_max(D^{-1}A) (30 Lanczos steps) is a
    lower bound within 2% of the exact value on every smoothing level."""
    n = 64
    P = eth.Problem(n)
    nlev, lam = P.levels()
    exact = _oracle_lambdas(n)
    assert nlev == len(exact) + 1
    for a, e in zip(lam, exact):
        assert e * 0.98 <= a <= e * (1 + 1e-8)


@pytest.mark.parametrize("use_graph", [False, True])
def test_solve_config1_exact_velocity_diag_mq(use_graph):
    """Stokes cavity 16 x 16, lid (1,0), f = 0, exact A, diagonal M_Q with the
    bordered projection, FP64 MINRES."""
    n = 16
    print(f"[solve c1] graph={use_graph}", flush=True)
    m = Mesh(n)
    s = System(m)
    b_ref = s.rhs(None, lid_dirichlet(m))
    xd = direct_solve(s, b_ref)
    P = eth.Problem(n, velocity=eth.VEL_EXACT, mq=eth.MQ_DIAG)
    b = P.assemble_rhs()
    x, info = P.solve(b, rtol=1e-12, maxit=3000, use_graph=use_graph, true_residual=True)
    assert info[0]["status"] == 0
    assert rel_err(_np(x), xd) < 1e-8
    # iteration count equals the oracle's MINRES with the same preconditioner
    Pref = _oracle_prec(s, "exact", "diag")
    _, oinfo = minres(lambda v: s.K @ v, s.to_interior(b_ref), Pref, tol=1e-12, maxit=3000)
    assert abs(info[0]["iterations"] - oinfo["iterations"]) <= 2
    # at the configured tolerance 1e-6
    x6, info6 = P.solve(b, rtol=1e-6, use_graph=use_graph)
    _, oinfo6 = minres(lambda v: s.K @ v, s.to_interior(b_ref), Pref, tol=1e-6, maxit=3000)
    assert abs(info6[0]["iterations"] - oinfo6["iterations"]) <= 1


@pytest.mark.parametrize("prec,tol_rel", [(eth.FP64, 1e-8), (eth.MIXED, 1e-6)])
def test_solve_gmg_cheb_sgs_matches_direct(prec, tol_rel):
    n = 64
    print(f"[solve gmg] n={n} prec={prec}", flush=True)
    m = Mesh(n)
    s = System(m)
    xd = direct_solve(s, s.rhs(None, lid_dirichlet(m)))
    P = eth.Problem(n, precision=prec)
    b = P.assemble_rhs()
    # an FP32 preconditioner limits the attainable MINRES accuracy, so the
    # mixed run stops at 1e-8 (or its iteration limit) and is held to 1e-6
    rtol = 1e-12 if prec == eth.FP64 else 1e-8
    x, info = P.solve(b, rtol=rtol, maxit=600, use_graph=True, true_residual=True)
    print(f"  iterations={info[0]['iterations']} status={info[0]['status']} "
          f"true_rel={info[0]['rel_residual_true']:.2e}", flush=True)
    assert info[0]["status"] in (0, eth.WMAXIT), info
    if prec == eth.FP64:
        assert info[0]["status"] == 0
    assert rel_err(_np(x), xd) < tol_rel


def test_solve_batched_forcing_matches_direct():
    n = 32
    B = 4
    m = Mesh(n)
    s = System(m)
    P = eth.Problem(n, max_batch=B, precision=eth.MIXED)
    F = torch.stack([_t(gaussian_bumps(n, 1000 + k)) for k in range(B)])
    b = P.assemble_rhs(F, batch=B)
    x, infos = P.solve(b, rtol=1e-8, maxit=600, use_graph=True)
    X = _np(x)
    for k in range(B):
        xd = direct_solve(s, s.rhs(gaussian_bumps(n, 1000 + k), lid_dirichlet(m)))
        assert infos[k]["status"] in (0, eth.WMAXIT)
        assert rel_err(X[k], xd) < 1e-6


def test_solve_x0_warm_start_and_zero_rhs():
    n = 16
    m = Mesh(n)
    s = System(m)
    P = eth.Problem(n, velocity=eth.VEL_EXACT, mq=eth.MQ_DIAG)
    b = P.assemble_rhs()
    xd = direct_solve(s, s.rhs(None, lid_dirichlet(m)))
    xl, _ = P.solve(b, rtol=1e-3, maxit=2000)
    x2, info2 = P.solve(b, rtol=1e-11, x0=xl)
    assert info2[0]["status"] == 0
    assert rel_err(_np(x2), xd) < 1e-8
    # zero right-hand side: x = 0 immediately
    z = torch.zeros_like(b)
    x0, i0 = P.solve(z, rtol=1e-8)
    assert i0[0]["iterations"] == 0 and float(x0.abs().max()) == 0.0


@pytest.mark.parametrize("n,velocity,mq", [(8, "exact", "diag"), (16, "exact", "diag"), (32, "gmg", "cheb_sgs")])
def test_est_minres_matches_oracle(n, velocity, mq):
    """The inf-sup estimate from the Lanczos scalars recorded on the device
    during the GPU solve against the oracle's estimate from its own MINRES
    with the same preconditioner (Sec. 2.4)."""
    from oracle.infsup import est_minres
    print(f"[est-minres] n={n} {velocity} {mq}", flush=True)
    m = Mesh(n)
    s = System(m)
    lam = _oracle_lambdas(n) if velocity == "gmg" else None
    P = eth.Problem(n, velocity=eth.VEL_GMG if velocity == "gmg" else eth.VEL_EXACT,
                    mq=eth.MQ_DIAG if mq == "diag" else eth.MQ_CHEB_SGS, gmg_lambda=lam,
                    mq_cheb=(_mq_lo(n), 1.0))
    b = P.assemble_rhs()
    _, info = P.solve(b, rtol=1e-10, maxit=3000)
    g2, th, k = P.infsup_estimate(0)
    bref = s.to_interior(s.rhs(None, lid_dirichlet(m)))
    _, oinfo = minres(lambda v: s.K @ v, bref, _oracle_prec(s, velocity, mq, lambdas=lam), tol=1e-10, maxit=3000)
    og2, oth = est_minres(oinfo["delta"], oinfo["gamma"])
    assert abs(k - oinfo["iterations"]) <= 1
    assert th < 0
    assert abs(g2 - og2) <= 1e-6 * og2


@pytest.mark.parametrize("n,prec,tol", [(16, eth.FP64, 1e-11), (64, eth.FP64, 1e-11), (64, eth.MIXED, 2e-5)])
def test_schur_gmg_preconditioner_matches_oracle(n, prec, tol):
    """M_Q^+ by elimination of the P0 block with a Q1 multigrid for S_k
    (the GPU's Lanczos bounds passed to the oracle)."""
    print(f"[schur mq] n={n} prec={prec}", flush=True)
    m = Mesh(n)
    nu = 0.5
    s = System(m, nu=nu)
    lam = _oracle_lambdas(n)
    P = eth.Problem(n, nu=nu, velocity=eth.VEL_GMG, mq=eth.MQ_SCHUR_GMG, precision=prec, gmg_lambda=lam)
    _, slam = P.q1_levels()
    r = uniform_vector(m.N, 21 + n)
    r[: 2 * m.nv][s.vel_bnd] = 0.0
    z = _np(P.apply_preconditioner(_t(r)))
    Pref = opc.StokesBlockDiag(s, "gmg", "schur_gmg", gmg_kw=dict(lambdas=lam), schur_kw=dict(lambdas=slam))
    zref = s.to_full(Pref(s.to_interior(r)))
    o = 2 * m.nv
    assert rel_err(z[:o], zref[:o]) < tol
    assert rel_err(z[o:], zref[o:]) < tol


@pytest.mark.parametrize("prec", [eth.FP64, eth.MIXED])
def test_schur_gmg_solve_is_mesh_independent(prec):
    """MINRES with the P0-elimination M_Q: iteration counts of the oracle with
    the same preconditioner (+-1) and mesh independent from 32^2 to 128^2."""
    its = []
    for n in (32, 64, 128):
        m = Mesh(n)
        s = System(m)
        P = eth.Problem(n, velocity=eth.VEL_GMG, mq=eth.MQ_SCHUR_GMG, precision=prec)
        b = P.assemble_rhs()
        x, info = P.solve(b, rtol=1e-6, true_residual=True)
        assert info[0]["status"] == 0
        its.append(info[0]["iterations"])
        if n == 64:
            _, slam = P.q1_levels()
            _, vlam = P.levels()
            Pref = opc.StokesBlockDiag(s, "gmg", "schur_gmg", gmg_kw=dict(lambdas=vlam),
                                       schur_kw=dict(lambdas=slam))
            _, oinfo = minres(lambda v: s.K @ v, s.to_interior(s.rhs(None, lid_dirichlet(m))), Pref,
                              tol=1e-6, maxit=1000)
            assert abs(info[0]["iterations"] - oinfo["iterations"]) <= 1
    print(f"  iterations {its}", flush=True)
    assert max(its) - min(its) <= 3


def test_sync_probes_run():
    """The persistent-kernel probe (grid-wide barriers in one cooperative
    launch) and the launch-boundary probe (graph-replayed dependent launches)
    both complete and report a per-step time."""
    P = eth.Problem(128)      # the probe borrows a workspace of 512 doubles per CU
    g, _ = P.profile_kernel(eth.K_SYNC_GRAPH, reps=200)
    c, _ = P.profile_kernel(eth.K_SYNC_GRID, reps=200)
    print(f"[sync probe] graph launch {1e3 * g:.2f} us, grid barrier {1e3 * c:.2f} us", flush=True)
    assert 0 < g < 1.0 and 0 < c < 1.0
    P.close()
