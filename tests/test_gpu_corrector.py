"""The corrected coarse step in the engine, and the restriction/set-up calls."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import cnn
from oracle import model_h as mh
from paper_0710_5912_amd import configs, inputs

pytestmark = pytest.mark.gpu

le = pytest.importorskip("paper_0710_5912_amd.le")


def test_restrict_is_block_mean():
    p = configs.model_h(64, 64, gdot=0.1)
    phi0 = inputs.noise_phi0(64, 64, 3, amp=0.5)
    om0 = inputs.noise_omega0(64, 64, 3)
    with le.Context(p, phi0, om0) as c:
        c.step(20)
        st = c.get_state()
        phi_c, om_c = c.restrict(4)
    assert np.max(np.abs(phi_c - cnn.restrict4(st["phi"]))) <= 1e-15
    assert np.max(np.abs(om_c - cnn.restrict4(st["omega"]))) <= 1e-15
    assert abs(phi_c.mean() - st["phi"].mean()) <= 1e-15


def test_set_fields_resolves_psi():
    p = configs.model_h(32, 32, gdot=0.2)
    phi0 = inputs.noise_phi0(32, 32, 4, amp=0.5)
    om0 = inputs.noise_omega0(32, 32, 4)
    with le.Context(p, np.zeros((32, 32))) as c:
        c.set_fields(phi0, om0, 137)
        g = c.get_state()
    op = mh.Params(**p)
    s = mh.strain_offset(op, 137)
    _, psi = mh.stage_flow(mh.Params(**dict(p, dt=0.0)), om0 - om0.mean(), np.zeros_like(om0), s)
    assert g["step"] == 137 and g["wraps"] == mh.wrap_count(op, 137)
    assert np.max(np.abs(g["psi"] - psi)) <= 1e-12 * np.max(np.abs(psi))


@pytest.mark.parametrize("scheme", [False, True])
def test_zero_network_leaves_the_plain_step(scheme):
    """With the last layer zeroed the residual vanishes: corrected = plain,
    also with the scheme switches on (they act on the corrected step's plain
    part as on the plain step)."""
    p = configs.model_h(64, 64, gdot=0.5, rho=1.0)
    phi0 = inputs.noise_phi0(64, 64, 5, amp=0.5)
    params = inputs.cnn_init_params(1)
    params[19104:] = 0.0
    with le.Context(p, phi0) as a, le.Context(p, phi0) as b:
        if scheme:
            a.set_scheme(f_half=True, midpoint_s=True)
            b.set_scheme(f_half=True, midpoint_s=True)
        a.corrector_load(params, [1.0, 10.0, 1.0, 1.0])
        a.step_corrected(220)          # crosses the wrap at strain 0.5 (step 200)
        b.step(220)
        ga, gb = a.get_state(), b.get_state()
    assert ga["wraps"] == gb["wraps"] == 1
    for k in ("phi", "omega", "psi"):
        assert np.max(np.abs(ga[k] - gb[k])) <= 1e-12 * np.max(np.abs(gb[k])), k


def projected(r0, projection):
    """The phi residual as the corrector adds it: minus its mean (mode 0) or
    minus its interpolated tile means (mode 1)."""
    return r0 - (r0.mean() if projection == 0 else cnn.tile_mean_field(r0))


@pytest.mark.parametrize("projection", [0, 1])
def test_corrected_step_applies_the_network(projection):
    """One corrected step = plain step + network residual (mean-free in phi)."""
    p = configs.model_h(64, 64, gdot=0.1, rho=1.0)
    phi0 = inputs.noise_phi0(64, 64, 6, amp=0.6)
    params = inputs.cnn_init_params(2) * 3.0
    scales = [1.0, 10.0, 0.05, 0.01]
    with le.Context(p, phi0) as a, le.Context(p, phi0) as b:
        a.corrector_load(params, scales)
        a.corrector_projection(projection)
        a.step_corrected(1)
        b.step(1)
        ga, gb = a.get_state(), b.get_state()
    x = np.stack([gb["phi"], gb["omega"]])
    rparams = np.concatenate([np.concatenate([cnn.bf16_round(Wl).ravel(),
                                              np.asarray(bb, np.float32).astype(np.float64)])
                              for Wl, bb in cnn.unpack(np.asarray(params, np.float32))])
    r = cnn.forward(rparams, x, scales, round_act=cnn.bf16_round)
    d_phi = ga["phi"] - gb["phi"]
    d_om = ga["omega"] - gb["omega"]
    assert abs(d_phi.mean()) <= 1e-15
    assert abs(ga["phi"].mean() - phi0.mean()) <= 1e-14
    assert np.max(np.abs(d_phi - projected(r[0], projection))) <= 2e-2 * np.max(np.abs(r[0]))
    assert np.max(np.abs(d_om - r[1])) <= 2e-2 * np.max(np.abs(r[1]))


@pytest.mark.parametrize("projection", [0, 1])
@pytest.mark.parametrize("n", [64, 256])
def test_fused_network_equals_the_layer_kernels(fixed_variants, n, projection):
    """The corrected step runs the network as one tiled kernel (activations in
    LDS, 4-pixel halos); its residual equals the per-layer kernels' output on
    the same planes (unit output scales: r = z exactly), up to the FP64 sum
    order of the mean."""
    torch = pytest.importorskip("torch")
    p = configs.model_h(n, n, gdot=0.1, rho=1.0)
    phi0 = inputs.noise_phi0(n, n, 9, amp=0.6)
    params = inputs.cnn_init_params(4) * 3.0
    scales = [1.0, 10.0, 1.0, 1.0]
    with le.Context(p, phi0) as a, le.Context(p, phi0) as b:
        a.corrector_load(params, scales)
        a.corrector_projection(projection)
        a.step_corrected(1)
        b.step(1)
        ga, gb = a.get_state(), b.get_state()
    net = le.Net(n, n)
    try:
        net.set_params(params, scales)
        x = torch.from_numpy(np.stack([gb["phi"], gb["omega"]]).astype(np.float32)[None]).cuda()
        r = torch.empty_like(x)
        net.forward(x, r)
        torch.cuda.synchronize()
        r = r.cpu().numpy()[0].astype(np.float64)
    finally:
        net.close()
    d_phi = ga["phi"] - gb["phi"]
    d_om = ga["omega"] - gb["omega"]
    assert np.max(np.abs(d_phi - projected(r[0], projection))) <= 1e-12 * np.max(np.abs(r[0]))
    assert np.max(np.abs(d_om - r[1])) <= 1e-12 * np.max(np.abs(r[1]))
    assert abs(d_phi.mean()) <= 1e-15


def test_projection_switch_reaches_captured_chunks_and_rejects_unknown_modes():
    """Switching the projection between graph-captured corrected chunks takes
    effect (the chunks are re-captured): 64 corrected steps in mode 1 after 64
    in mode 0 equal a context that ran the same sequence uncaptured, in
    profiled calls; mode 2 is rejected."""
    p = configs.model_h(64, 64, gdot=0.1, rho=1.0)
    phi0 = inputs.noise_phi0(64, 64, 7, amp=0.5)
    params = inputs.cnn_init_params(3)
    scales = [1.0, 10.0, 0.05, 0.01]
    with le.Context(p, phi0) as a, le.Context(p, phi0) as b:
        for c in (a, b):
            c.corrector_load(params, scales)
        b.profile(True)
        for mode in (0, 1):
            for c in (a, b):
                c.corrector_projection(mode)
                c.step_corrected(64)
        ga, gb = a.get_state(), b.get_state()
        assert le.lib().le_corrector_projection(a._h, 2) == le.LE_EINVAL
    for k in ("phi", "omega", "psi"):
        assert np.max(np.abs(ga[k] - gb[k])) <= 1e-12 * np.max(np.abs(gb[k])), k


def test_corrector_needs_inertia_and_a_load():
    p = configs.model_h(32, 32, rho=0.0)
    with le.Context(p, inputs.noise_phi0(32, 32, 0)) as c:
        with pytest.raises(le.LeError):
            c.corrector_load(inputs.cnn_init_params(0), [1, 1, 1, 1])
    p = configs.model_h(32, 32, rho=1.0)
    with le.Context(p, inputs.noise_phi0(32, 32, 0)) as c:
        with pytest.raises(le.LeError):
            c.step_corrected(1)


def test_corrected_graph_replays_match_eager(fixed_variants):
    monkeypatch = fixed_variants
    """Corrected chunks replayed from a captured graph equal direct launches,
    replay after replay, and a reload with new scales is not replayed stale."""
    p = configs.model_h(64, 64, gdot=0.1, rho=1.0)
    phi0 = inputs.noise_phi0(64, 64, 8, amp=0.6)
    params = inputs.cnn_init_params(3) * 2.0
    a = le.Context(p, phi0)
    monkeypatch.setenv("LE_GRAPHS", "0")
    b = le.Context(p, phi0)
    monkeypatch.delenv("LE_GRAPHS")
    try:
        for scales in ([1.0, 10.0, 0.02, 0.005], [0.5, 5.0, 0.04, 0.001]):
            a.corrector_load(params, scales)
            b.corrector_load(params, scales)
            for rep in range(3):
                a.step_corrected(16)
                b.step_corrected(16)
                ga, gb = a.get_state(), b.get_state()
                for k in ("phi", "omega", "psi"):
                    assert np.array_equal(ga[k], gb[k]), (scales, rep, k)
    finally:
        a.close()
        b.close()


def test_audit_that_passes_leaves_the_corrected_run(fixed_variants):
    """Audits every 10 corrected steps (windows of 4) with a tolerance no run
    exceeds: the state equals the unaudited corrected run bit for bit."""
    p = configs.model_h(64, 64, gdot=0.1, rho=1.0)
    phi0 = inputs.noise_phi0(64, 64, 8, amp=0.6)
    params = inputs.cnn_init_params(3) * 2.0
    scales = [1.0, 10.0, 0.02, 0.005]
    with le.Context(p, phi0) as a, le.Context(p, phi0) as b:
        a.corrector_load(params, scales)
        b.corrector_load(params, scales)
        a.corrector_audit(10, 4, 1e9)
        a.step_corrected(30)
        b.step_corrected(30)
        ga, gb = a.get_state(), b.get_state()
        fallback, audits, dev = a.corrector_status()
    assert ga["step"] == gb["step"] == 30
    for k in ("phi", "omega", "psi"):
        assert np.max(np.abs(ga[k] - gb[k])) <= 1e-12 * np.max(np.abs(gb[k])), k
    assert not fallback and audits == 2 and 0.0 < dev < 1e9


def test_failed_audit_falls_back_to_plain_steps(fixed_variants):
    """With tolerance 0 the first audit (steps 6..8) fails: the context keeps
    the plain result of that window and steps plainly from then on, so the run
    equals 6 corrected steps followed by 14 plain ones, bit for bit."""
    p = configs.model_h(64, 64, gdot=0.1, rho=1.0)
    phi0 = inputs.noise_phi0(64, 64, 9, amp=0.6)
    params = inputs.cnn_init_params(4) * 2.0
    scales = [1.0, 10.0, 0.02, 0.005]
    with le.Context(p, phi0) as a, le.Context(p, phi0) as b:
        a.corrector_load(params, scales)
        b.corrector_load(params, scales)
        a.corrector_audit(6, 3, 0.0)
        a.step_corrected(20)
        fallback, audits, dev = a.corrector_status()
        b.step_corrected(6)
        b.step(14)
        ga, gb = a.get_state(), b.get_state()
        assert fallback and audits == 1 and dev > 0.0
        a.corrector_audit(0, 0, 0.0)
        assert a.corrector_status() == (False, 0, 0.0)
        with pytest.raises(le.LeError) as ei:
            a.corrector_audit(5, 0, 0.02)
        assert ei.value.code == le.LE_EINVAL
    assert ga["step"] == gb["step"] == 20
    for k in ("phi", "omega", "psi"):
        assert np.max(np.abs(ga[k] - gb[k])) <= 1e-12 * np.max(np.abs(gb[k])), k


def test_audit_needs_a_corrector():
    p = configs.model_h(32, 32, rho=1.0)
    with le.Context(p, inputs.noise_phi0(32, 32, 0)) as c:
        with pytest.raises(le.LeError) as ei:
            c.corrector_audit(10, 2, 0.02)
        assert ei.value.code == le.LE_EINVAL


def test_stage_timing_of_long_corrected_calls_without_graphs(monkeypatch):
    """Stage timing on and graphs off: corrected calls longer than the timing
    event pool run in pieces that fit it, count every corrected step's stages,
    and give the same state as an untimed run."""
    monkeypatch.setenv("LE_GRAPHS", "0")
    p = configs.model_h(64, 64, gdot=0.1, rho=1.0)
    phi0 = inputs.noise_phi0(64, 64, 8, amp=0.5)
    params = inputs.cnn_init_params(3)
    scales = [1.0, 10.0, 0.05, 0.01]
    with le.Context(p, phi0) as a, le.Context(p, phi0) as b:
        for c in (a, b):
            c.corrector_load(params, scales)
        a.profile(True)
        a.step_corrected(300)
        b.step_corrected(300)
        times = a.stage_times()
        ga, gb = a.get_state(), b.get_state()
    assert all(n == 300 for _, n in times.values()), times
    assert all(ms > 0.0 for ms, _ in times.values()), times
    for k in ("phi", "omega", "psi"):
        assert np.max(np.abs(ga[k] - gb[k])) <= 1e-12 * np.max(np.abs(gb[k])), k
