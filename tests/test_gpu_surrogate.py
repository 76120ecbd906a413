"""The learned Front2VOF surrogate end to end: training rows from the
method's own runs, training on the GPU kernels, the gain over the untrained
network and over a colour-count estimate, and its use inside Front2VOF
(ambiguous cells exactly geometric, the others exactly the network)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from oracle import mlp_oracle as M
from paper_2509_26361_amd import ebit as E
from paper_2509_26361_amd import inputs as I
from paper_2509_26361_amd import surrogate as SG

pytestmark = pytest.mark.gpu


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def interfacial(flags):
    """Flat mask of the cells with a marker on one of their 12 edges."""
    n = flags.shape[0]
    f = flags.ravel()
    cells = np.arange(n ** 3)
    x, y, z = cells % n, (cells // n) % n, cells // (n * n)
    out = np.zeros(n ** 3, bool)
    for e in range(3):
        others = [a for a in range(3) if a != e]
        for oA in (0, 1):
            for oB in (0, 1):
                off = [0, 0, 0]
                off[others[0]], off[others[1]] = oA, oB
                q = (x + off[0]) % n + n * (((y + off[1]) % n) + n * ((z + off[2]) % n))
                out |= ((f[q] >> (4 + e)) & 1) == 1
    return out


def test_dataset_rows_match_oracle_features_and_labels():
    """Rows of ebit_surrogate_dataset = the oracle's features and geometric
    volume fractions of the unambiguous interfacial cells."""
    n = 32
    st = O.init(I.random_shape(n, 12), exact=True)
    e = E.Ebit(n, "fp64", dev())
    e.load_state(T(st.flags), [T(x) for x in st.s])
    C = torch.zeros((n, n, n), dtype=torch.float64, device=dev())
    e.front2vof(C)
    X, c = e.dataset()
    Co, amb = O.f2v(st)
    want = np.nonzero(interfacial(st.flags) & (amb.ravel() == 0))[0]
    assert X.shape[0] == len(want) and len(want) > 500
    assert torch.all(X[:, 20:] == 0)
    got = np.c_[X.float().cpu().numpy()[:, :20].astype(np.float64), c.cpu().numpy().astype(np.float64)]
    ref = np.c_[M.bf16(M.cell_features(st.flags, st.s, want)), Co.ravel()[want].astype(np.float32)]
    key = lambda a: a[np.lexsort(a.T[::-1])]
    assert np.array_equal(key(got), key(ref))
    # the labels agree with the GPU's own geometric Front2VOF
    assert np.array_equal(np.sort(c.cpu().numpy()), np.sort(C.cpu().numpy().ravel()[want].astype(np.float32)))


def test_trained_surrogate_gains_and_front2vof_integration():
    X, c = SG.make_dataset(n=64, shapes=6, snapshots=3, seed=1, device=dev())
    Xh, ch = SG.make_dataset(n=64, shapes=2, snapshots=2, seed=99, device=dev())
    print(f"rows: train {X.shape[0]}, held out {Xh.shape[0]}")
    assert X.shape[0] > 5000 and Xh.shape[0] > 1000
    theta0 = torch.from_numpy(I.mlp_init(3).astype(np.float32)).to(dev())
    mae0, _ = SG.evaluate(theta0, Xh, ch)
    theta = SG.train(X, c, steps=1500, batch=2048, lr=3e-3, seed=3, theta=theta0.clone())
    mae, mx = SG.evaluate(theta, Xh, ch)
    naive = float((Xh[:, 12:20].float().mean(dim=1) - ch).abs().mean().item())   # phase-1 corner fraction
    print(f"held-out MAE: trained {mae:.4f} (max {mx:.3f}), untrained {mae0:.4f}, corner fraction {naive:.4f}")
    assert mae < 0.25 * mae0
    assert mae < 0.5 * naive

    # a deformed sphere (few ambiguous cells) and a random interface (many)
    n = 64
    sh = I.sphere_shape(n, centre=(0.5, 0.5, 0.5), R=0.27)
    e = E.Ebit(n, "fp64", dev())
    e.init(T(sh.phi_nodes), [T(f) for f in sh.phi_faces])
    U = [T(u) for u in I.deformation_velocity(n)]
    for k in range(40):
        e.step(U, I.deformation_time_factor(k * 0.5 / n, 3.0), 0.5 / n)
    check_in_front2vof(e, n, theta, vol_tol=1e-2)
    n = 32
    st = O.init(I.random_shape(n, 21), exact=True)
    e = E.Ebit(n, "fp64", dev())
    e.load_state(T(st.flags), [T(x) for x in st.s])
    U = [T(u) for u in I.fourier_velocity(n, seed=22, modes=3)]
    for k in range(3):
        e.step(U, 1.0, 0.5 / n)
    assert check_in_front2vof(e, n, theta, vol_tol=3e-2) > 0


def check_in_front2vof(e, n, theta, vol_tol):
    """Front2VOF with the surrogate = geometric on cells without markers and
    on ambiguous cells, the network's output on the others; returns the
    number of ambiguous cells."""
    Cg = torch.zeros((n, n, n), dtype=torch.float64, device=dev())
    e.front2vof(Cg)
    assert e.stats(Cg)["n_surrogate"] == 0
    Xr, cr = e.dataset()
    e.set_surrogate(theta)
    Cs = torch.zeros_like(Cg)
    e.front2vof(Cs)                                           # a new C: every cell recomputed
    n_surrogate = e.stats(Cs)["n_surrogate"]
    e.set_surrogate(None)
    fl, s = e.state()
    st = O.State(n, fl.cpu().numpy(), [x.cpu().numpy() for x in s])
    _, amb = O.f2v(st)
    amb = amb.ravel().astype(bool)
    inter = interfacial(st.flags)
    Cg_, Cs_ = Cg.cpu().numpy().ravel(), Cs.cpu().numpy().ravel()
    assert np.array_equal(Cs_[~inter], Cg_[~inter])           # full / empty cells
    assert np.array_equal(Cs_[amb], Cg_[amb])                 # ambiguous cells: geometric
    y = E.mlp_forward(theta, Xr).double().cpu().numpy()
    assert np.array_equal(np.sort(Cs_[inter & ~amb]), np.sort(y))   # the others: the network
    assert n_surrogate == int((inter & ~amb).sum()) == len(y)
    vg, vs = Cg_.sum(), Cs_.sum()
    print(f"n={n}: {int(amb.sum())} ambiguous, {int(inter.sum())} interfacial; volume geometric {vg:.3f}, "
          f"surrogate {vs:.3f}, rel diff {abs(vs - vg) / vg:.2e}")
    assert abs(vs - vg) / vg < vol_tol
    return int(amb.sum())


def test_output_bias_calibration_matches_mean_label():
    """After calibrate_bias the network's mean output on the calibration rows
    equals their mean label (Newton on the output bias); only b3 changes."""
    rng = np.random.default_rng(3)
    m = 20000
    feats = np.concatenate([rng.uniform(0, 1, (m, 12)) * (rng.uniform(0, 1, (m, 12)) < 0.3),
                            (rng.uniform(0, 1, (m, 8)) < 0.5).astype(np.float64), np.zeros((m, 12))], axis=1)
    X = T(feats.astype(np.float32)).to(torch.bfloat16).contiguous()
    c = T(rng.uniform(0.2, 0.9, m).astype(np.float32))
    theta = T(I.mlp_init(5).astype(np.float32))
    before = float(E.mlp_forward(theta, X).double().mean().item())
    th2, d = SG.calibrate_bias(theta, X, c)
    after = float(E.mlp_forward(th2, X).double().mean().item())
    target = float(c.double().mean().item())
    assert abs(before - target) > 1e-2           # there was a bias to remove
    assert abs(after - target) < 2e-5, (after, target, d)
    assert torch.equal(th2[:-1], theta[:-1]) and float(th2[-1] - theta[-1]) == pytest.approx(d, abs=1e-6)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_advance_with_surrogate_fused_equals_separate_launches(prec):
    """With the surrogate set, ebit_advance puts the classify pass of each
    Front2VOF into the next x sweep's launch and runs the network's pass
    after it.  Against EBIT_OPT_FUSE off and against single calls (sweeps,
    then ebit_front2vof): state, C and counters bit-identical, at a ragged
    brick count.  The network is a seeded untrained one (the test is about
    the launches)."""
    n = 44
    dtype = torch.float64 if prec == "fp64" else torch.float32
    sh = I.sphere_shape(n, centre=(0.45, 0.5, 0.55), R=0.2)
    U = [T(u).to(dtype) for u in I.deformation_velocity(n)]
    theta = torch.from_numpy(I.mlp_init(5).astype(np.float32)).to(dev())
    dt = 0.5 / n
    gs = [I.deformation_time_factor(k * dt, 3.0) for k in range(9)]
    out = []
    for mode in ("fused", "unfused", "calls"):
        e = E.Ebit(n, prec, dev())
        e.init(T(sh.phi_nodes), [T(f) for f in sh.phi_faces])
        e.set_surrogate(theta)
        C = torch.zeros((n, n, n), dtype=dtype, device=dev())
        if mode == "calls":
            for g in gs:
                e.step(U, g, dt)
                e.front2vof(C)
        else:
            e.set_option(E.EBIT_OPT_FUSE, 1 if mode == "fused" else 0)
            e.advance(U, gs, dt, C)
        torch.cuda.synchronize()
        fl, s = e.state()
        out.append((fl.clone(), [x.clone() for x in s], C.clone(), e.stats(C)))
    f0, s0, c0, st0 = out[0]
    assert st0["n_interfacial"] > 0
    for f1, s1, c1, st1 in out[1:]:
        assert torch.equal(f0, f1)
        for k in range(3):
            assert torch.equal(s0[k], s1[k])
        assert torch.equal(c0, c1)
        for key in ("n_interfacial", "n_interfacial_sum", "n_ambiguous", "n_markers"):
            assert st0[key] == st1[key], key


def test_trained_surrogate_against_geometric_front2vof():
    """What the trained network gains or loses against the geometric
    Front2VOF it replaces, on the same FP32 run (C does not feed back into
    the advection, so both runs hold the same state at every step): the
    state bit-identical, the network's error on the unambiguous interfacial
    cells (mean below 0.01, volume within 1e-3), and the step time of each,
    printed as the ratio."""
    X, c = SG.make_dataset(n=64, shapes=8, snapshots=3, seed=4, device=dev())
    theta = SG.train(X, c, steps=3000, batch=4096, lr=3e-3, seed=5,
                     theta=torch.from_numpy(I.mlp_init(6).astype(np.float32)).to(dev()))
    n, steps = 128, 120
    sh = I.sphere_shape(n)
    U = [T(u).float() for u in I.deformation_velocity(n)]
    dt = 0.5 / n
    gs = [I.deformation_time_factor(k * dt, 3.0) for k in range(steps)]
    runs = {}
    for mode in ("geometric", "surrogate"):
        e = E.Ebit(n, "fp32", dev())
        e.init(T(sh.phi_nodes), [T(f) for f in sh.phi_faces])
        if mode == "surrogate":
            e.set_surrogate(theta)
        C = torch.zeros((n, n, n), dtype=torch.float32, device=dev())
        e.front2vof(C)
        e.advance(U, gs[:20], dt, C)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        e.advance(U, gs[20:], dt, C)
        b.record()
        torch.cuda.synchronize()
        fl, s = e.state()
        runs[mode] = (fl.clone(), [x.clone() for x in s], C.clone(), a.elapsed_time(b) / (steps - 20))
    (fg, sg, Cg, tg), (fs, ss, Cs, ts) = runs["geometric"], runs["surrogate"]
    assert torch.equal(fg, fs)
    for k in range(3):
        assert torch.equal(sg[k], ss[k])
    mixed = (Cg > 0) & (Cg < 1)
    diff = (Cs - Cg).abs()[mixed].double()
    vol = abs(float(Cs.double().sum() - Cg.double().sum())) / float(Cg.double().sum())
    print(f"surrogate vs geometric Front2VOF at {n}^3 (FP32): mean |dC| {float(diff.mean()):.2e}, "
          f"max {float(diff.max()):.2e}, volume {vol:.2e}; ms/step {ts:.4f} vs {tg:.4f} (x{ts / tg:.2f})")
    assert float(diff.mean()) < 1e-2
    assert vol < 1e-3
    assert tg > 0 and ts > 0
