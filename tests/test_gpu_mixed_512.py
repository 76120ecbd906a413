"""The large mixed workload at full size: 512^3, 4096 seeded spheres (radii
3..12 cells) in a seeded divergence-free Fourier field, CFL 0.5, run by
ebit_advance with its defaults for this size (brick-ordered lists, waves on
contiguous runs of them, sparse task loads, Front2VOF fused with the next x
sweep).

The oracle cannot take a step of this grid in seconds.  What holds at any
size is checked instead:
- the run equals, bit for bit, the same run with lists in claim order and
  the same steps issued as single calls, whose bands take all neighbours
  (the kernels whose oracle parity the smaller tests establish);
- the state is consistent: an edge carries a marker exactly where its end
  colours differ (sec. 2.2), and every fraction lies in [0, 1);
- the interfacial-cell counter agrees with the flags."""
import numpy as np
import pytest
import torch

from paper_2509_26361_amd import ebit as E
from paper_2509_26361_amd import inputs as I

pytestmark = pytest.mark.gpu
N = 512
STEPS = 12


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def workload():
    d = dev()
    free, total = torch.cuda.mem_get_info(d)
    if total < 64 * 2**30:
        pytest.skip("needs a GPU with about 40 GB")
    cs, rs = I.random_nonoverlapping_spheres(4096, 3.0, 12.0, N, gap_cells=2.0, seed=0)
    sh = I.spheres_shape(N, cs, rs, with_s=False)
    phi = torch.from_numpy(sh.phi_nodes).to(d)
    pf = [torch.from_numpy(f).to(d) for f in sh.phi_faces]
    del sh
    U = I.fourier_velocity_device(N, seed=1, modes=8, device=d)
    return phi, pf, U


def run(workload, order, prec="fp64", theta=None, calls=False):
    """The run through ebit_advance, or (calls) one call per sweep and per
    Front2VOF, where no sweep knows the next one's axis (all 26 neighbours
    join the band)."""
    phi, pf, U = workload
    dtype = torch.float64 if prec == "fp64" else torch.float32
    e = E.Ebit(N, prec, dev())
    e.init(phi, pf)
    if order is not None:
        e.set_option(E.EBIT_OPT_ORDER, order)
    if theta is not None:
        e.set_surrogate(theta)
    C = torch.zeros((N, N, N), dtype=dtype, device=dev())
    e.front2vof(C)
    Ud = [u.to(dtype) for u in U]
    if calls:
        for _ in range(STEPS):
            e.step(Ud, 1.0, 0.5 / N)
            e.front2vof(C)
    else:
        e.advance(Ud, [1.0] * STEPS, 0.5 / N, C)
    torch.cuda.synchronize()
    return e, C


def test_mixed_512_ordered_run_equals_claim_order_and_is_consistent(workload):
    a, Ca = run(workload, None)           # the default at this size: ordered
    fa, sa = a.state()
    st_a = a.stats(Ca)
    b, Cb = run(workload, 0)
    fb, sb = b.state()
    assert torch.equal(fa, fb)
    for k in range(3):
        assert torch.equal(sa[k], sb[k]), k
    assert torch.equal(Ca, Cb)
    st_b = b.stats(Cb)
    for key in ("n_interfacial", "n_interfacial_sum", "n_fallback", "n_cfl", "volume", "volume_comp"):
        assert st_a[key] == st_b[key], key
    del b, Cb, fb, sb
    torch.cuda.empty_cache()
    # single calls: the band without the next axis known
    c, Cc = run(workload, None, calls=True)
    fc, sc = c.state()
    assert torch.equal(fa, fc)
    for k in range(3):
        assert torch.equal(sa[k], sc[k]), k
    assert torch.equal(Ca, Cc)
    del c, Cc, fc, sc
    torch.cuda.empty_cache()

    # edge markers exactly where the end colours differ (x fastest: tensor dim 2 - e)
    col = fa & 1
    for e in range(3):
        m = (fa >> (4 + e)) & 1
        differ = (col != torch.roll(col, -1, 2 - e)).to(torch.uint8)
        assert torch.equal(m, differ), f"axis {e}: {int((m != differ).sum())} inconsistent edges"
        s = sa[e][m.bool()]
        assert bool(((s >= 0) & (s < 1)).all()), f"axis {e}: fraction outside [0, 1)"
    assert st_a["n_cfl"] == 0
    # interfacial cells: a marker on any of the cell's 12 edges
    has = torch.zeros_like(col, dtype=torch.bool)
    for e in range(3):
        m = ((fa >> (4 + e)) & 1).bool()
        a1, a2 = [2 - x for x in range(3) if x != e]
        has |= m | torch.roll(m, -1, a1) | torch.roll(m, -1, a2) | torch.roll(torch.roll(m, -1, a1), -1, a2)
    assert st_a["n_interfacial"] == int(has.sum())
    assert st_a["n_interfacial"] > 4_000_000


@pytest.mark.parametrize("surrogate", [False, True])
def test_mixed_512_fp32_forms_ordered_equal_claim_order(workload, surrogate):
    """The FP32 form, and the FP32 form with the surrogate (a seeded untrained
    network: the test is about the lists, not the network), at full size:
    ordered lists bit-identical to claim order."""
    theta = torch.from_numpy(I.mlp_init(3).astype(np.float32)).to(dev()) if surrogate else None
    a, Ca = run(workload, None, "fp32", theta)
    fa, sa = a.state()
    b, Cb = run(workload, 0, "fp32", theta)
    fb, sb = b.state()
    assert torch.equal(fa, fb)
    for k in range(3):
        assert torch.equal(sa[k], sb[k]), k
    assert torch.equal(Ca, Cb)
    assert a.stats(Ca)["n_interfacial_sum"] == b.stats(Cb)["n_interfacial_sum"]


def test_mixed_512_step_against_oracle(workload):
    """Oracle parity at full size in the default launch configuration
    (brick-ordered lists, runs, sparse task loads, directional band, fused
    Front2VOF): after STEPS GPU steps the state goes to the oracle, both take
    one more step (three sweeps, then Front2VOF), and every node and cell is
    compared -- flags bit-exact, fractions and C within 1e-12."""
    from oracle import oracle as O
    phi, pf, U = workload
    e = E.Ebit(N, "fp64", dev())
    e.init(phi, pf)
    C = torch.zeros((N, N, N), dtype=torch.float64, device=dev())
    e.front2vof(C)
    e.advance(U, [1.0] * STEPS, 0.5 / N, C)
    torch.cuda.synchronize()
    fl, s = e.state()
    st = O.State(N, fl.cpu().numpy().copy(), [x.cpu().numpy() for x in s])
    e.advance(U, [1.0], 0.5 / N, C)
    torch.cuda.synchronize()
    Uh = [u.cpu().numpy() for u in U]
    st, cnt = O.step(st, Uh, 1.0, 0.5 / N)
    del Uh
    assert cnt[0] == 0 and cnt[2] == 0
    fl, s = e.state()
    f = fl.cpu().numpy()
    bad = np.argwhere(f != st.flags)
    assert len(bad) == 0, f"{len(bad)} flag mismatches, first at {bad[:3].tolist()}"
    del f
    for k in range(3):
        d = float(np.max(np.abs(s[k].cpu().numpy() - st.s[k])))
        assert d <= 1e-12, f"s[{k}] differs by {d}"
    Co, _ = O.f2v(st)
    d = float(np.max(np.abs(C.cpu().numpy() - Co)))
    assert d <= 1e-12, f"C differs by {d}"
    del Co
    # the refinement band of this state (sec. 2.3) against its oracle
    from oracle import refine as Rf
    mask, bricks, counts = E.refine_band(fl)
    wm = Rf.refine_mask(st.flags)
    assert np.array_equal(mask.cpu().numpy(), wm.astype(np.uint8))
    assert np.array_equal(bricks.cpu().numpy(), Rf.refine_bricks(wm).astype(np.uint8))
    assert counts.cpu().tolist()[:2] == [int(Rf.interfacial(st.flags).sum()), int(wm.sum())]
