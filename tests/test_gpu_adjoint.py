"""GPU checks of the hand-written adjoint of the coupled step, through the C ABI.

* one reverse step == the oracle's autograd vector-Jacobian product (FP64,
  element by element, 1e-10 relative);
* a checkpointed rollout's gradient w.r.t. zeta, q0 and the initial Q field ==
  the oracle's autograd gradient of the same rollout (FP64);
* the 32^3 droplet (R = 8, q0 = 2 pi/12, zeta = 0.006), 400 steps with
  checkpoints every 20: adjoint gradients vs FP64 central differences
  (h = 1e-6) on zeta, q0 and 10 Q entries inside the droplet, within 1e-4
  relative (FP64 and FP32 adjoints).
"""
import math

import numpy as np
import pytest
import torch

from oracle import core
from paper_2011_00287_amd import inputs
from paper_2011_00287_amd.autograd import backward_segments, displacement_loss, run_segments
from paper_2011_00287_amd.sim import Sim

from helpers import rel_err

pytestmark = pytest.mark.gpu
DT = torch.float64


def _p(**kw):
    return dict(inputs.BASE_PARAMS, **kw)


@pytest.mark.parametrize("shape", [(6, 5, 7), (9, 8, 4)])
def test_single_step_vjp_matches_oracle(shape):
    nx, ny, nz = shape
    p = _p(q0=2 * math.pi / 7, zeta=0.01)
    g, phi, q5 = inputs.random_fields(nx, ny, nz, seed=31 + nx, g_amp=2e-3, q_amp=0.2)
    rng = np.random.default_rng(5)
    ab_g = rng.normal(size=g.shape)
    ab_q = rng.normal(size=q5.shape)
    ab_p = rng.normal(size=phi.shape)
    # oracle: autograd of <a_bar, step(x)>
    gt = torch.tensor(g, requires_grad=True)
    qt = torch.tensor(q5, requires_grad=True)
    pt = torch.tensor(phi, requires_grad=True)
    zt = torch.tensor(p["zeta"], dtype=DT, requires_grad=True)
    q0t = torch.tensor(p["q0"], dtype=DT, requires_grad=True)
    po = dict(p, zeta=zt, q0=q0t)
    go, qo, pho = core.step(gt, qt, pt, po)
    s = (go * torch.tensor(ab_g)).sum() + (qo * torch.tensor(ab_q)).sum() + (pho * torch.tensor(ab_p)).sum()
    s.backward()
    # GPU
    with Sim(p, phi, q5, precision="fp64") as sim:
        sim.set_fields(g=g)
        state = sim.get_state()
        adj = sim.adjoint_buffer()
        bg, bq, bp = sim.adjoint_parts(adj)
        bg.copy_(torch.tensor(ab_g))
        bq.copy_(torch.tensor(ab_q))
        bp.copy_(torch.tensor(ab_p))
        out = sim.adjoint_buffer()
        zb, qb = sim.adjoint_step(state, adj, out)
        # the same step with a recorded u, F instead of the recomputation
        rec = sim.record_buffer()
        nxt = torch.empty_like(state)
        sim.step_record(state, nxt, rec)
        out2 = sim.adjoint_buffer()
        zb2, qb2 = sim.adjoint_step(state, adj, out2, rec=rec)
        # the recorded u, F come from the fused kernels, the recomputed ones from the
        # site kernels: equal up to float64 rounding of differently ordered sums
        assert float((out - out2).abs().max()) <= 1e-13 * float(out.abs().max())
        assert abs(zb2 - zb) <= 1e-13 * abs(zb) and abs(qb2 - qb) <= 1e-13 * abs(qb)
        # the recorded step equals an ordinary step (state buffers hold padding: compare fields)
        sim.set_state(state)
        sim.step(1)
        ref = sim.moments() + (sim.populations(),)
        sim.set_state(nxt)
        for a, b in zip(ref, sim.moments() + (sim.populations(),)):
            assert np.array_equal(a, b)
        sim.set_state(state)
        bg, bq, bp = (t.cpu().numpy() for t in sim.adjoint_parts(out))
    for name, a, b in (("g", bg, gt.grad.numpy()), ("q", bq, qt.grad.numpy()), ("phi", bp, pt.grad.numpy())):
        l2, mx = rel_err(a, b)
        assert l2 < 1e-10 and mx < 1e-10, (name, l2, mx)
    assert abs(zb - float(zt.grad)) <= 1e-10 * abs(float(zt.grad))
    assert abs(qb - float(q0t.grad)) <= 1e-10 * abs(float(q0t.grad))


def _oracle_rollout_grad(p, phi, q5, steps):
    qt = torch.tensor(q5, requires_grad=True)
    zt = torch.tensor(p["zeta"], dtype=DT, requires_grad=True)
    q0t = torch.tensor(p["q0"], dtype=DT, requires_grad=True)
    po = dict(p, zeta=zt, q0=q0t)
    phit = torch.tensor(phi)
    zc0 = core.centre_linear(phit)[2].detach()
    g = torch.zeros((19,) + phi.shape, dtype=DT)
    g, q, ph = core.run(g, qt, phit, po, steps)
    L = core.displacement_loss(ph, zc0)
    L.backward()
    return float(L.detach()), float(zt.grad), float(q0t.grad), qt.grad.numpy()


def test_rollout_gradient_matches_oracle_autograd():
    p = _p(q0=2 * math.pi / 8, zeta=0.02)
    phi, q5 = inputs.droplet_fields(8, 8, 10, 2.5, p["q0"], seed=3)
    steps = 7
    L_o, dz_o, dq0_o, dq5_o = _oracle_rollout_grad(p, phi, q5, steps)
    zeta = torch.tensor(p["zeta"], dtype=DT, requires_grad=True)
    q0 = torch.tensor(p["q0"], dtype=DT, requires_grad=True)
    q5t = torch.tensor(q5, requires_grad=True)
    L = displacement_loss(zeta, q0, q5t, params=p, phi=phi, steps=steps, checkpoint=3, precision="fp64")
    L.backward()
    # L is the square of a small difference of centres: rounding is amplified
    assert abs(float(L.detach()) - L_o) <= 1e-10 * abs(L_o)
    assert abs(float(zeta.grad) - dz_o) <= 1e-9 * abs(dz_o)
    assert abs(float(q0.grad) - dq0_o) <= 1e-9 * abs(dq0_o)
    l2, mx = rel_err(q5t.grad.numpy(), dq5_o)
    assert l2 < 1e-9 and mx < 1e-9, (l2, mx)


def _loss_fwd(p, phi, q5, steps, precision="fp64"):
    with Sim(p, phi, q5, precision=precision) as s:
        zc0 = s.centre()[0][2]
        s.step(steps)
        zc = s.centre()[0][2]
    return (zc - zc0) ** 2


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-5), ("fp32", 1e-4)])
def test_droplet32_adjoint_vs_central_differences(precision, tol):
    w = inputs.WORKLOADS["droplet32_adjoint"]
    p = inputs.params_for("droplet32_adjoint")
    phi, q5 = inputs.workload_fields("droplet32_adjoint")
    steps, ck = w["steps"], w["checkpoint"]
    # adjoint gradients
    with Sim(p, phi, q5, precision=precision) as sim:
        zc0 = sim.centre()[0][2]
        ckpts = run_segments(sim, steps, ck)
        adj = sim.adjoint_buffer()
        L = sim.seed_centre(zc0, adj)
        dz, dq0 = backward_segments(sim, ckpts, steps, ck, adj)
        _, qbar, _ = sim.adjoint_parts(adj)
        qbar = qbar.double().cpu().numpy()
    assert L > 0
    # FP64 central differences: with h = 1e-6 their own rounding noise after 400
    # steps is ~1e-12 absolute on gradients of ~1e-6, i.e. ~1e-6 relative.
    h = 1e-6
    fd_z = (_loss_fwd(dict(p, zeta=p["zeta"] + h), phi, q5, steps) -
            _loss_fwd(dict(p, zeta=p["zeta"] - h), phi, q5, steps)) / (2 * h)
    fd_q0 = (_loss_fwd(dict(p, q0=p["q0"] + h), phi, q5, steps) -
             _loss_fwd(dict(p, q0=p["q0"] - h), phi, q5, steps)) / (2 * h)
    assert abs(dz - fd_z) <= tol * abs(fd_z), (dz, fd_z)
    assert abs(dq0 - fd_q0) <= tol * abs(fd_q0), (dq0, fd_q0)
    # 10 Q entries inside the droplet (phi > phi_cr), drawn with seed 0
    rng = np.random.default_rng(0)
    inside = np.argwhere(phi > p["phi_cr"])
    picks = inside[rng.choice(len(inside), 10, replace=False)]
    comps = rng.integers(0, 5, 10)
    def fd_q(c, z, y, x, hh):
        qp = q5.copy()
        qm = q5.copy()
        qp[c, z, y, x] += hh
        qm[c, z, y, x] -= hh
        return (_loss_fwd(p, phi, qp, steps) - _loss_fwd(p, phi, qm, steps)) / (2 * hh)

    ads, fds, fds2 = [], [], []
    for (z, y, x), c in zip(picks, comps):
        fds.append(fd_q(c, z, y, x, h))
        fds2.append(fd_q(c, z, y, x, 2 * h))
        ads.append(qbar[c, z, y, x])
    ads, fds, fds2 = np.array(ads), np.array(fds), np.array(fds2)
    # each entry on its own, at the 1e-4 relative bar, plus a floor for the noise of
    # the difference quotients: measured as their change from h to 2h (the O(h^2)
    # truncation is far below it), times 3; float32 adds its own rounding of the
    # reverse sweep, 1e-5 of the largest gradient
    noise = np.abs(fds - fds2).max()
    floor = 3 * noise + (1e-5 * np.abs(fds).max() if precision == "fp32" else 0.0)
    ratio = np.abs(ads - fds) / (1e-4 * np.abs(fds) + floor)
    print(precision, "Q entries: ad", ads, "fd", fds, "fd noise", noise, "worst |ad - fd| / bound", ratio.max())
    assert np.all(ratio <= 1.0), (ads, fds, ratio)


def test_parameter_sums_kept_on_device_between_fetches():
    """Reverse steps that leave the zeta / q0 sums on the device, fetched once at
    the end, give the same totals (to float64 rounding) as fetching every step;
    a fetch clears the device sums."""
    p = _p(q0=2 * math.pi / 7, zeta=0.01)
    g, phi, q5 = inputs.random_fields(7, 6, 5, seed=11, g_amp=2e-3, q_amp=0.2)
    rng = np.random.default_rng(9)
    with Sim(p, phi, q5, precision="fp64") as sim:
        sim.set_fields(g=g)
        states = [sim.get_state()]
        for _ in range(3):
            sim.step(1)
            states.append(sim.get_state())
        seed = sim.adjoint_buffer()
        seed.copy_(torch.tensor(rng.normal(size=seed.numel())))

        def sweep(fetch_every):
            cur, nxt = seed.clone(), sim.adjoint_buffer()
            zb = qb = 0.0
            for j in (2, 1, 0):
                zb, qb = sim.adjoint_step(states[j], cur, nxt, zeta_bar=zb, q0_bar=qb, fetch=fetch_every or j == 0)
                cur, nxt = nxt, cur
            return zb, qb, cur

        z1, q1, a1 = sweep(True)
        z2, q2, a2 = sweep(False)
        z3, q3, _ = sweep(True)  # nothing left over from the previous sweep
    assert torch.equal(a1, a2)
    for a, b in ((z1, z2), (q1, q2), (z1, z3), (q1, q3)):
        assert abs(a - b) <= 1e-13 * abs(a), (a, b)
    assert z1 != 0.0 and q1 != 0.0


def test_recorded_rollout_equals_checkpointed():
    """checkpoint = 0 keeps the lean record of every step instead of replaying
    segments.  The reverse collision then takes u and rho - rho0 from the
    forward kernel's record rather than recomputing them from the populations,
    so the gradients agree to float64 rounding, not bit for bit."""
    p = _p(q0=2 * math.pi / 8, zeta=0.02)
    phi, q5 = inputs.droplet_fields(8, 8, 10, 2.5, p["q0"], seed=3)
    grads = []
    for ck in (3, 0):
        zeta = torch.tensor(p["zeta"], dtype=DT, requires_grad=True)
        q0 = torch.tensor(p["q0"], dtype=DT, requires_grad=True)
        q5t = torch.tensor(q5, requires_grad=True)
        L = displacement_loss(zeta, q0, q5t, params=p, phi=phi, steps=7, checkpoint=ck, precision="fp64")
        L.backward()
        grads.append((float(L.detach()), float(zeta.grad), float(q0.grad), q5t.grad.numpy()))
    (L1, z1, c1, g1), (L2, z2, c2, g2) = grads
    assert L1 == L2
    assert abs(z1 - z2) <= 1e-12 * abs(z1) and abs(c1 - c2) <= 1e-12 * abs(c1)
    l2, mx = rel_err(g2, g1)
    assert l2 < 1e-12 and mx < 1e-12, (l2, mx)


@pytest.mark.parametrize("shape", [(34, 18, 11), (33, 9, 5), (12, 6, 7), (64, 16, 5), (64, 40, 6)])
@pytest.mark.parametrize("tz", ["1", "3", "default"])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 1e-5)])
@pytest.mark.parametrize("adj_tile", [1, 2])
def test_adjoint_site_and_tiled_kernels_agree(prec, tol, tz, shape, adj_tile):
    """The site-parallel and the z-marching tiled reverse kernels (the order kernel
    and the fused stress + gather kernel with its tile-face terms) give the same
    reverse step, for several slab depths.  Boxes: ragged tiles and slabs
    (34 x 18 x 11); edge tiles one column and one row wide, whose sites send
    across both faces of an axis (33 x 9 x 5); one tile smaller than the tile
    shape, which wraps periodically inside itself (12 x 6 x 7); whole tiles
    only, on two or more x tiles and two y tiles (64 x 16 x 5); three 16-row
    tiles and a ragged one (64 x 40 x 6).  Both tile heights of the stress and
    order adjoints (8 and 16 rows)."""
    p = _p(q0=2 * math.pi / 9, zeta=0.01)
    g, phi, q5 = inputs.random_fields(*shape, seed=21, g_amp=2e-3, q_amp=0.2)
    seed_vals = np.random.default_rng(4).normal(size=25 * phi.size)
    tz_adj = 0 if tz == "default" else int(tz)
    outs = []
    for path in ("default", "site"):
        with Sim(p, phi, q5, precision=prec, tuning={"path": path, "tz_adj": tz_adj, "adj_tile": adj_tile,
                                                              "adj_order_tile": adj_tile}) as sim:
            sim.set_fields(g=g)
            state = sim.get_state()
            adj = sim.adjoint_buffer()
            adj.copy_(torch.tensor(seed_vals, dtype=adj.dtype))
            out = sim.adjoint_buffer()
            zb, qb = sim.adjoint_step(state, adj, out)
            outs.append((out.double().cpu().numpy(), zb, qb))
    (a, za, qa), (b, zb_, qb_) = outs
    l2, mx = rel_err(a, b)
    assert l2 < tol and mx < tol, (l2, mx)
    assert abs(za - zb_) <= tol * abs(za) and abs(qa - qb_) <= tol * abs(qa)


@pytest.mark.parametrize("shape", [(290, 20, 4), (20, 290, 4)])
def test_adjoint_tiled_kernels_on_lines_longer_than_a_face_block(shape):
    """Rows (columns) longer than the 256 lines one block of the face fix-up
    covers, with a two-column (four-row) last tile: the tiled reverse equals
    the site-parallel one in FP64."""
    p = _p(q0=2 * math.pi / 9, zeta=0.01)
    g, phi, q5 = inputs.random_fields(*shape, seed=23, g_amp=2e-3, q_amp=0.2)
    seed_vals = np.random.default_rng(5).normal(size=25 * phi.size)
    outs = []
    for path in ("default", "site"):
        with Sim(p, phi, q5, precision="fp64", tuning={"path": path}) as sim:
            sim.set_fields(g=g)
            state = sim.get_state()
            adj = sim.adjoint_buffer()
            adj.copy_(torch.tensor(seed_vals, dtype=adj.dtype))
            out = sim.adjoint_buffer()
            zb, qb = sim.adjoint_step(state, adj, out)
            outs.append((out.double().cpu().numpy(), zb, qb))
    (a, za, qa), (b, zb_, qb_) = outs
    l2, mx = rel_err(a, b)
    assert l2 < 1e-13 and mx < 1e-13, (l2, mx)
    assert abs(za - zb_) <= 1e-13 * abs(za) and abs(qa - qb_) <= 1e-13 * abs(qa)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 1e-5)])
def test_lean_reverse_step_equals_full_state_step(prec, tol):
    """The reverse of a step from its lean record (Q, phi, drho, u, F) equals the reverse
    from the full state and its u, F, drho record (the populations enter only through drho, u)."""
    p = _p(q0=2 * math.pi / 7, zeta=0.01)
    g, phi, q5 = inputs.random_fields(9, 8, 6, seed=41, g_amp=2e-3, q_amp=0.2)
    seed_vals = np.random.default_rng(6).normal(size=25 * phi.size)
    with Sim(p, phi, q5, precision=prec) as sim:
        sim.set_fields(g=g)
        state = sim.get_state()
        adj = sim.adjoint_buffer()
        adj.copy_(torch.tensor(seed_vals, dtype=adj.dtype))
        rec = sim.record_buffer()
        nxt = torch.empty_like(state)
        sim.step_record(state, nxt, rec)
        out_full = sim.adjoint_buffer()
        zf, qf = sim.adjoint_step(state, adj, out_full, rec=rec)
        sim.set_state(state)
        lean = sim.lean_record_buffer()
        assert lean.numel() < state.numel() + rec.numel() * rec.element_size()
        sim.step_record_lean(lean)
        assert sim.totals()["step"] == 1
        # the lean recording step advanced the context exactly as an ordinary step
        sim2_ref = sim.moments()
        sim.set_state(nxt)
        for a, b in zip(sim2_ref, sim.moments()):
            assert np.array_equal(a, b)
        out_lean = sim.adjoint_buffer()
        zl, ql = sim.adjoint_step_lean(lean, adj, out_lean)
    a, b = out_lean.double().cpu().numpy(), out_full.double().cpu().numpy()
    l2, mx = rel_err(a, b)
    assert l2 < tol and mx < tol, (l2, mx)
    assert abs(zl - zf) <= tol * abs(zf) and abs(ql - qf) <= tol * abs(qf)


def test_lean_rollouts_equal_full_state_rollout():
    """run_lean + backward_lean and the lean checkpointed replay give the gradient of the
    full-state checkpointed rollout (FP64)."""
    from paper_2011_00287_amd.autograd import backward_lean, backward_segments_lean, run_lean
    p = _p(q0=2 * math.pi / 8, zeta=0.02)
    phi, q5 = inputs.droplet_fields(10, 9, 12, 3.0, p["q0"], seed=5)
    steps, ck = 11, 4
    res = []
    for mode in ("full", "lean", "lean_ckpt"):
        with Sim(p, phi, q5, precision="fp64") as sim:
            zc0 = sim.centre()[0][2]
            if mode == "lean":
                recs = run_lean(sim, steps)
            else:
                ckpts = run_segments(sim, steps, ck)
            adj = sim.adjoint_buffer()
            L = sim.seed_centre(zc0, adj)
            if mode == "full":
                zb, qb = backward_segments(sim, ckpts, steps, ck, adj)
            elif mode == "lean":
                zb, qb = backward_lean(sim, recs, adj)
            else:
                zb, qb = backward_segments_lean(sim, ckpts, steps, ck, adj)
            res.append((L, zb, qb, adj.double().cpu().numpy()))
    (L0, z0, q0_, a0) = res[0]
    for L, zb, qb, a in res[1:]:
        assert abs(L - L0) <= 1e-14 * abs(L0)
        assert abs(zb - z0) <= 1e-12 * abs(z0) and abs(qb - q0_) <= 1e-12 * abs(q0_)
        l2, mx = rel_err(a, a0)
        assert l2 < 1e-12 and mx < 1e-12, (l2, mx)


def test_lean_records_refused_without_adjoint():
    """A context without an adjoint (the pc4 integrator on the site-parallel test
    kernels) has no lean records either."""
    from paper_2011_00287_amd._lib import LB_EINVAL, LbError
    phi, q5 = inputs.droplet_fields(6, 6, 6, 2.0, 0.5)
    with Sim(_p(M=0.05), phi, q5, fd_scheme="pc4", tuning={"path": "site"}) as sim:
        assert sim.lean_record_buffer().numel() == 0
        with pytest.raises(LbError) as e:
            sim.step_record_lean(torch.empty(8, dtype=torch.uint8, device="cuda"))
        assert e.value.status == LB_EINVAL


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_overlapped_replay_equals_sequential(prec):
    """Replaying segment s-1 on a second context and stream while segment s is reversed
    gives the sequential checkpointed sweep bit for bit."""
    from paper_2011_00287_amd.autograd import backward_segments_overlapped
    p = _p(q0=2 * math.pi / 8, zeta=0.02)
    phi, q5 = inputs.droplet_fields(12, 10, 14, 3.5, p["q0"], seed=7)
    steps, ck = 13, 4
    res = []
    replay_stream = torch.cuda.Stream()
    for mode in ("sequential", "overlapped"):
        with Sim(p, phi, q5, precision=prec, stream=torch.cuda.current_stream()) as sim:
            zc0 = sim.centre()[0][2]
            ckpts = run_segments(sim, steps, ck)
            adj = sim.adjoint_buffer()
            sim.seed_centre(zc0, adj)
            if mode == "sequential":
                zb, qb = backward_segments(sim, ckpts, steps, ck, adj)
            else:
                with Sim(p, phi, q5, precision=prec, stream=replay_stream) as rep:
                    zb, qb = backward_segments_overlapped(sim, rep, ckpts, steps, ck, adj, replay_stream)
            torch.cuda.synchronize()
            res.append((zb, qb, adj.cpu().numpy().copy()))
    assert res[0][0] == res[1][0] and res[0][1] == res[1][1]
    assert np.array_equal(res[0][2], res[1][2])


@pytest.mark.parametrize("adj_tile", [1, 2])
def test_fp64_reverse_with_16_plane_slabs_equals_site_kernels(adj_tile):
    """The reverse step with 16-plane slabs of both adjoint marches (the slab depth of the benchmark's
    128^3 box), on a box whose last slabs are ragged, against the site-parallel reverse kernels."""
    p = _p(q0=2 * math.pi / 9, zeta=0.01)
    g, phi, q5 = inputs.random_fields(40, 24, 36, seed=31, g_amp=2e-3, q_amp=0.2)
    seed_vals = np.random.default_rng(5).normal(size=25 * phi.size)
    outs = []
    for tuning in ({"tz_adj": 16, "tz_adj_order": 16, "adj_tile": adj_tile, "adj_order_tile": adj_tile},
                   {"path": "site"}):
        with Sim(p, phi, q5, precision="fp64", tuning=tuning) as sim:
            sim.set_fields(g=g)
            state = sim.get_state()
            adj = sim.adjoint_buffer()
            adj.copy_(torch.tensor(seed_vals, dtype=adj.dtype))
            out = sim.adjoint_buffer()
            zb, qb = sim.adjoint_step(state, adj, out)
            outs.append((out.cpu().numpy(), zb, qb))
    (a, za, qa), (b, zb_, qb_) = outs
    l2, mx = rel_err(a, b)
    assert l2 < 1e-13 and mx < 1e-13, (l2, mx)
    assert abs(za - zb_) <= 1e-13 * abs(za) and abs(qa - qb_) <= 1e-13 * abs(qa)
