"""GPU path (through the C ABI) against the FP64 oracle, element by element.

Bar: FP64 fields within 1e-10 relative (max norm over the field) of the
oracle after 100 steps on the same seeded inputs; observables within 1e-12
relative.  FP32 runs are held to the bound derived in the design notes.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import model_h as mh
from oracle import observables as ob
from paper_0710_5912_amd import inputs

pytestmark = pytest.mark.gpu

le = pytest.importorskip("paper_0710_5912_amd.le")


def params(nx, ny, **kw):
    base = dict(nx=nx, ny=ny, lx=float(nx), ly=float(ny), gdot=0.01, A=1.0, B=1.0,
                kappa=1.0, M=1.0, eta=1.0, rho=1.0, dt=0.005)
    base.update(kw)
    return base


def rel(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def run_pair(p, steps, seed=0, amp=0.05, omega=False, precision="fp64"):
    phi0 = inputs.noise_phi0(p["ny"], p["nx"], seed, amp=amp)
    om0 = inputs.noise_omega0(p["ny"], p["nx"], seed) if omega else None
    print(f"case nx={p['nx']} ny={p['ny']} gdot={p['gdot']} rho={p['rho']} "
          f"steps={steps} seed={seed} {precision}", flush=True)
    ctx = le.Context(p, phi0, om0, precision=precision)
    ctx.step(steps)
    g = ctx.get_state()
    op = mh.Params(**p)
    st = mh.run(op, mh.initial_state(op, phi0, om0), steps)
    return ctx, g, st, op


@pytest.mark.parametrize("rho", [1.0, 0.0])
def test_small_case_fp64_100_steps(rho):
    """64x64, gdot = 0.01, dt = 0.005: the small workload, 100 steps."""
    p = params(64, 64, rho=rho)
    ctx, g, st, _ = run_pair(p, 100)
    assert g["step"] == 100 and g["wraps"] == st.wraps
    assert rel(g["phi"], st.phi) <= 1e-10
    assert rel(g["psi"], st.psi) <= 1e-10
    if rho > 0:
        assert rel(g["omega"], st.omega) <= 1e-10
    ctx.close()


@pytest.mark.parametrize("nx,ny,lx,ly,gdot,rho", [
    (32, 16, 2.0, 1.0, 8.0, 1.0),     # c = r = 2 (the paper's geometry), one wrap
    (16, 16, 16.0, 16.0, -6.0, 1.0),  # negative shear, c = r = 1
    (64, 16, 4.0, 1.0, 12.0, 0.0),    # r = 4, Stokes branch
    (8, 8, 8.0, 8.0, 3.0, 1.0),       # the smallest grid
])
def test_parity_through_strain_wraps(nx, ny, lx, ly, gdot, rho):
    p = params(nx, ny, lx=lx, ly=ly, gdot=gdot, rho=rho, kappa=0.05 * (lx / nx) ** 2 * 20,
               M=0.5 * (lx / nx) ** 2, dt=0.002)
    ctx, g, st, op = run_pair(p, 100, omega=True, amp=0.5)
    assert st.wraps != 0
    assert g["wraps"] == st.wraps
    assert rel(g["phi"], st.phi) <= 1e-10
    assert rel(g["psi"], st.psi) <= 1e-10
    if rho > 0:
        assert rel(g["omega"], st.omega) <= 1e-10
    ctx.close()


@pytest.mark.parametrize("nx,ny", [(128, 64), (256, 128), (64, 256), (512, 32)])
def test_parity_several_tiles(nx, ny):
    """Grids spanning several row/column blocks, ragged final column block."""
    p = params(nx, ny, gdot=0.0 if nx < ny else 0.05, rho=1.0)
    ctx, g, st, _ = run_pair(p, 40, seed=3, omega=True)
    assert rel(g["phi"], st.phi) <= 1e-10
    assert rel(g["omega"], st.omega) <= 1e-10
    assert rel(g["psi"], st.psi) <= 1e-10
    ctx.close()


def test_observables_match_oracle():
    p = params(64, 32, lx=128.0, ly=64.0, gdot=0.3, rho=2.0)
    ctx, g, st, op = run_pair(p, 150, seed=5, amp=0.6, omega=True)
    o, Sk = ctx.observables()
    ro, rSk, _ = ob.observables(op, st)
    for k in ("mean_phi", "phi2", "Ls", "Dxx", "Dxy", "Dyy", "L_perp", "L_par", "sigma_xy",
              "sigma_xy_re", "s", "strain", "t"):
        a, b = o[k], ro[k]
        if math.isinf(b):
            assert math.isinf(a) or a > 1e12, (k, a, b)
            continue
        assert abs(a - b) <= 1e-12 * max(abs(b), 1e-300) + 1e-18, (k, a, b)
    assert o["step"] == ro["step"] and o["wraps"] == ro["wraps"]
    assert o["finite"] == 1 and o["nbins"] == 16
    assert np.max(np.abs(Sk - rSk)) <= 1e-12 * np.max(np.abs(rSk))
    ctx.close()


def test_mean_phi_conserved_and_deterministic(fixed_variants):
    p = params(128, 128, gdot=0.2, rho=1.0)
    phi0 = inputs.noise_phi0(128, 128, 9, amp=0.3, mean=0.1)
    runs = []
    for _ in range(2):
        ctx = le.Context(p, phi0)
        ctx.step(500)
        runs.append(ctx.get_state())
        o, _ = ctx.observables(sk=False)
        assert abs(o["mean_phi"] - float(np.mean(phi0))) <= 1e-13
        ctx.close()
    assert np.array_equal(runs[0]["phi"], runs[1]["phi"])
    assert np.array_equal(runs[0]["psi"], runs[1]["psi"])


@pytest.mark.parametrize("rho,prec", [(1.0, "fp64"), (0.0, "fp64"), (1.0, "fp32")])
def test_checkpoint_resume_is_bitwise(fixed_variants, rho, prec):
    """A blob saved at step 150 and loaded into a fresh context continues
    bit for bit as the run it came from (a wrap at step 200 in between)."""
    p = params(64, 64, gdot=1.0, rho=rho)
    phi0 = inputs.noise_phi0(64, 64, 2, amp=0.5)
    with le.Context(p, phi0, precision=prec) as a, \
            le.Context(p, np.zeros((64, 64)), precision=prec) as b:
        a.step(150)
        blob = a.checkpoint()
        a.step(150)
        ref = a.get_state()
        b.restore(blob)
        b.step(150)
        got = b.get_state()
        assert got["step"] == ref["step"] == 300 and got["wraps"] == ref["wraps"]
        for k in ("phi", "omega", "psi"):
            assert np.array_equal(got[k], ref[k]), k
        with pytest.raises(le.LeError) as ei:
            b.restore(blob[:-8])
        assert ei.value.code == le.LE_EINVAL
        # a blob of another spectral layout (the header's tile width, the
        # int32 after magic, version, nx, ny, precision and inertia)
        bad = bytearray(blob)
        bad[28:32] = (int.from_bytes(blob[28:32], "little") + 1).to_bytes(4, "little")
        with pytest.raises(le.LeError) as ei:
            b.restore(bytes(bad))
        assert ei.value.code == le.LE_EINVAL


def test_set_state_resume_to_rounding(fixed_variants):
    p = params(64, 64, gdot=1.0, rho=1.0)    # a wrap at strain 0.5 (step 100)
    phi0 = inputs.noise_phi0(64, 64, 2, amp=0.5)
    a = le.Context(p, phi0)
    a.step(150)
    mid = a.get_state()
    a.step(150)
    ref = a.get_state()
    b = le.Context(p, np.zeros((64, 64)))
    b.set_state(mid["phi"], mid["omega"], mid["psi"], mid["step"], mid["wraps"])
    b.step(150)
    got = b.get_state()
    assert got["step"] == 300 and got["wraps"] == ref["wraps"]
    # the restart rebuilds the row spectra from real fields: equal to rounding
    assert rel(got["phi"], ref["phi"]) <= 1e-13
    assert rel(got["psi"], ref["psi"]) <= 1e-12
    a.close()
    b.close()


def test_nonfinite_state_is_reported():
    p = params(32, 32)
    phi0 = inputs.noise_phi0(32, 32, 1)
    phi0[3, 4] = np.nan
    ctx = le.Context(p, phi0)
    with pytest.raises(le.LeError) as ei:
        ctx.step(2)
    assert ei.value.code == le.LE_ENONFINITE
    ctx.close()


@pytest.mark.parametrize("gdot", [0.0, 0.4])
def test_recovery_stops_at_the_last_finite_step(fixed_variants, gdot):
    """An explicit Cahn-Hilliard number of ~20 (dt = 1, kappa = 0.01) blows the
    run up (with gdot = 0.4 the strain wraps at step 2, inside the replay).
    With recovery on, the failing call leaves the context at the last step
    whose phi is finite: it equals a fresh run of that many steps bit for bit
    (same kernel variants, same wrap count), and one more step from there goes
    non-finite."""
    p = params(32, 32, gdot=gdot, kappa=0.01, dt=1.0)
    phi0 = inputs.noise_phi0(32, 32, 7, amp=0.05)
    with le.Context(p, phi0) as a, le.Context(p, phi0) as b:
        a.set_recovery(True)
        with pytest.raises(le.LeError) as ei:
            a.step(500)
        assert ei.value.code == le.LE_ENONFINITE
        g = a.get_state()
        m = g["step"]
        assert 0 < m < 500 and np.all(np.isfinite(g["phi"]))
        b.step(m)
        gb = b.get_state()
        assert g["wraps"] == gb["wraps"]
        for k in ("phi", "omega", "psi"):
            assert np.array_equal(g[k], gb[k], equal_nan=True), k
        with pytest.raises(le.LeError) as ei:
            b.step(1)
        assert ei.value.code == le.LE_ENONFINITE


def test_zero_steps_is_a_no_op_and_negative_steps_are_rejected():
    """le_step(c, 0) leaves the state, step counter and clock alone; a negative
    count is LE_EINVAL and changes nothing either."""
    p = params(32, 32, gdot=0.4)
    phi0 = inputs.noise_phi0(32, 32, 9, amp=0.3)
    with le.Context(p, phi0) as ctx:
        ctx.step(3)
        before = ctx.get_state()
        ctx.step(0)
        with pytest.raises(le.LeError) as ei:
            ctx.step(-1)
        assert ei.value.code == le.LE_EINVAL
        after = ctx.get_state()
        assert after["step"] == before["step"] == 3
        for k in ("phi", "omega", "psi"):
            assert np.array_equal(before[k], after[k]), k
        ctx.step(2)
        g = ctx.get_state()
    op = mh.Params(**p)
    st = mh.run(op, mh.initial_state(op, phi0), 5)
    assert rel(g["phi"], st.phi) <= 1e-10


@pytest.mark.parametrize("rho", [1.0, 0.0])
def test_fp32_error_bound(rho):
    """FP32 bulk: error after 100 steps stays within the stated 2e-5 bound."""
    p = params(64, 64, rho=rho)
    ctx, g, st, _ = run_pair(p, 100, precision="fp32")
    assert rel(g["phi"], st.phi) <= 2e-5
    assert rel(g["psi"], st.psi) <= 2e-4
    ctx.close()


def test_graph_replays_match_eager_launches(fixed_variants):
    monkeypatch = fixed_variants
    """Captured step graphs replayed many times, with eager work between the
    replays, give bit-identical states to plain launches."""
    p = params(128, 64, lx=256.0, ly=128.0, gdot=0.5, rho=1.0)   # wraps every 200 steps
    phi0 = inputs.noise_phi0(64, 128, 4, amp=0.5)
    monkeypatch.setenv("LE_GRAPHS", "0")
    eager = le.Context(p, phi0)
    monkeypatch.setenv("LE_GRAPHS", "1")
    graph = le.Context(p, phi0)
    for _ in range(6):
        eager.step(50)
        graph.step(50)
        a, b = eager.get_state(), graph.get_state()
        assert a["step"] == b["step"] and a["wraps"] == b["wraps"]
        for k in ("phi", "omega", "psi"):
            assert np.array_equal(a[k], b[k]), k
        oa, _ = eager.observables()
        ob_, _ = graph.observables()
        assert oa["Ls"] == ob_["Ls"]
    eager.close()
    graph.close()


def test_graph_pieces_of_irregular_chunks_match_eager_launches(fixed_variants):
    """Calls of irregular lengths (chunks cut at wraps and at the 128-step cap,
    replayed as power-of-two graph pieces) equal plain launches bit for bit,
    also against the oracle."""
    monkeypatch = fixed_variants
    p = params(64, 32, lx=128.0, ly=64.0, gdot=1.0, rho=1.0)   # wraps at steps 200, 600, 1000
    phi0 = inputs.noise_phi0(32, 64, 6, amp=0.5)
    monkeypatch.setenv("LE_GRAPHS", "0")
    eager = le.Context(p, phi0)
    monkeypatch.setenv("LE_GRAPHS", "1")
    graph = le.Context(p, phi0)
    for n in (37, 128, 5, 200, 77, 1, 300, 255):
        eager.step(n)
        graph.step(n)
        a, b = eager.get_state(), graph.get_state()
        assert a["step"] == b["step"] and a["wraps"] == b["wraps"]
        for k in ("phi", "omega", "psi"):
            assert np.array_equal(a[k], b[k]), (n, k)
    eager.close()
    graph.close()
    op = mh.Params(**p)
    st = mh.run(op, mh.initial_state(op, phi0), b["step"])
    assert st.wraps == b["wraps"] > 0
    assert rel(b["phi"], st.phi) <= 1e-10


@pytest.mark.parametrize("kw", [
    dict(A=0.7, B=1.3, kappa=4.0, M=2.0, eta=0.5, rho=2.0),
    dict(kappa=16.0, M=16.0),
    dict(A=0.7, B=1.3, kappa=4.0, M=2.0, eta=3.0, rho=0.0),
])
def test_parity_other_material_parameters(kw):
    """Free-energy, mobility, viscosity and density constants other than 1."""
    p = params(64, 64, gdot=0.05, **kw)
    ctx, g, st, _ = run_pair(p, 100, seed=5, amp=0.3)
    assert rel(g["phi"], st.phi) <= 1e-10
    assert rel(g["psi"], st.psi) <= 1e-10
    if kw.get("rho", 1.0) > 0:
        assert rel(g["omega"], st.omega) <= 1e-10
    ctx.close()


def test_long_run_statistics_fp64_and_fp32():
    """8000 steps (t = 40, domains formed and sheared) at 128^2: L(t),
    <phi^2> and the Korteweg stress of the FP64 and FP32 GPU runs against
    the oracle every 1000 steps, within 2% (the ensemble-statistics bar)."""
    from oracle import observables as ob
    p = params(128, 128, gdot=0.02, rho=1.0)
    phi0 = inputs.noise_phi0(128, 128, 5, amp=0.05)
    op = mh.Params(**p)
    st = mh.initial_state(op, phi0)
    ctx = {prec: le.Context(p, phi0, precision=prec) for prec in ("fp64", "fp32")}
    print("case 128^2 gdot=0.02 8000 steps, fp64 and fp32 vs oracle", flush=True)
    try:
        for k in range(8):
            st = mh.run(op, st, 1000)
            ro = ob.observables(op, st, 64)[0]
            if k < 3:
                continue          # before t = 20 the domains are still forming
            for prec, c in ctx.items():
                c.step(1000 if k > 3 else 4000)
                o, _ = c.observables(sk=False)
                assert o["step"] == st.step
                for key in ("Ls", "phi2"):
                    assert abs(o[key] - ro[key]) <= 0.02 * abs(ro[key]), (prec, k, key)
                assert abs(o["sigma_xy"] - ro["sigma_xy"]) <= 0.02 * abs(ro["sigma_xy"]) + 1e-9, \
                    (prec, k)
    finally:
        for c in ctx.values():
            c.close()
