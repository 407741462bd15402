"""Map and pose updates on the GPU against the float64 oracle, step by step
from the same float32 state.  adam_step: tensor sizes with ragged tails, a
tensor whose start is not 16-byte aligned (element-wise path), an empty
tensor, and more than one launch's worth of tensors.  pose_update: 53
sessions (two launches), four steps."""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_06644_amd import optim, rtgs
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

REL = 1e-5        # on the update p' - p (float32 division, square root, FMA)
U = 2.0 ** -24    # float32 unit roundoff


def _check_group(p_in, g, m_in, v_in, t, lr, b1, b2, eps, p_out, m_out, v_out):
    """Float32 error model: m is a two-term sum that may cancel, so its bound
    is a few roundings of the summands' magnitudes; v's terms never cancel;
    p' carries m's error times lr / (bias1 * denom), plus the update's own
    rounding and the final rounding of p'."""
    p_ref, m_ref, v_ref = oracle.adam_step(p_in, g, m_in, v_in, t, lr, b1, b2, eps)
    g64, m64 = g.astype(np.float64), m_in.astype(np.float64)
    m_bound = 4 * U * (b1 * np.abs(m64) + (1 - b1) * np.abs(g64)) + 1e-37
    assert np.all(np.abs(m_out - m_ref) <= m_bound), float(np.max(np.abs(m_out - m_ref) - m_bound))
    np.testing.assert_allclose(v_out, v_ref, rtol=8 * U, atol=1e-37)
    denom = np.sqrt(v_ref / (1 - b2 ** t)) + eps
    delta = np.abs(p_ref - p_in.astype(np.float64))
    bound = U * np.abs(p_ref) + REL * delta + lr / (1 - b1 ** t) / denom * m_bound + 1e-37
    assert np.all(np.abs(p_out - p_ref) <= bound), float(np.max(np.abs(p_out - p_ref) - bound))


def _run(sizes, steps, seed, b1=0.9, b2=0.999, eps=1e-8, misalign=()):
    h = rtgs.Handle(0)
    gen = torch.Generator(device="cuda").manual_seed(seed)
    groups = []
    for k, n in enumerate(sizes):
        off = 1 if k in misalign else 0
        mk = lambda: torch.randn(n + off, device="cuda", generator=gen)[off:]
        p = mk()
        m = torch.zeros(n + off, device="cuda")[off:]
        v = torch.zeros(n + off, device="cuda")[off:]
        groups.append([p, m, v, 10.0 ** (-2 - k % 3)])
    for t in range(1, steps + 1):
        grads = [torch.randn(len(gr[0]), device="cuda", generator=gen)
                 * 10.0 ** float(k % 5 - 2) for k, gr in enumerate(groups)]
        before = [[x.cpu().numpy() for x in gr[:3]] for gr in groups]
        rtgs.adam_step(h, [(p, g, m, v, lr, t) for (p, m, v, lr), g in zip(groups, grads)],
                       b1, b2, eps)
        torch.cuda.synchronize()
        for (p, m, v, lr), g, (p0, m0, v0) in zip(groups, grads, before):
            _check_group(p0, g.cpu().numpy(), m0, v0, t, lr, b1, b2, eps,
                         p.cpu().numpy(), m.cpu().numpy(), v.cpu().numpy())


def test_adam_ragged_sizes_and_unaligned_start():
    say("test_adam_ragged_sizes_and_unaligned_start")
    _run([0, 1, 3, 1023, 1024, 1025, 4097, 300_003, 5, 777], steps=3, seed=1, misalign=(4, 8, 9))


def test_adam_more_groups_than_one_launch():
    say("test_adam_more_groups_than_one_launch")
    rng = np.random.default_rng(2)
    _run([int(x) for x in rng.integers(1, 3000, size=70)], steps=2, seed=2, b1=0.8, b2=0.99,
         eps=1e-15, misalign=(3, 64))


def test_map_adam_many_sessions_equals_one_at_a_time():
    say("test_map_adam_many_sessions_equals_one_at_a_time")
    h = rtgs.Handle(0)
    gen = torch.Generator(device="cuda").manual_seed(3)
    shapes = [(1000, 3), (1000, 3), (1000, 4), (1000,), (1000, 3)]
    a = [[torch.randn(s, device="cuda", generator=gen) for s in shapes] for _ in range(2)]
    b = [[x.clone() for x in ps] for ps in a]
    oa = [optim.MapAdam(ps) for ps in a]
    ob = [optim.MapAdam(ps) for ps in b]
    for _ in range(3):
        gs = [[torch.randn(s, device="cuda", generator=gen) for s in shapes] for _ in range(2)]
        optim.step_many(h, list(zip(oa, gs)))
        for o, g in zip(ob, gs):
            o.step(h, g)
    torch.cuda.synchronize()
    for pa, pb in zip(a, b):
        for x, y in zip(pa, pb):
            assert torch.equal(x, y)
    assert oa[0].t == ob[1].t == 3


def test_adam_rejects_bad_arguments():
    say("test_adam_rejects_bad_arguments")
    h = rtgs.Handle(0)
    p = torch.zeros(8, device="cuda")
    for kw, t in ((dict(), 0), (dict(beta1=1.0), 1), (dict(eps=-1.0), 1)):
        with pytest.raises(rtgs.RtgsError) as e:
            rtgs.adam_step(h, [(p, p.clone(), p.clone(), p.clone(), 1e-3, t)], **kw)
        assert e.value.code == rtgs.RTGS_ERR_INVALID_ARG


def test_pose_update_matches_oracle_over_steps():
    say("test_pose_update_matches_oracle_over_steps")
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(11)
    n = 53                                            # more than one launch (48 per launch)
    vms, gs, ms, vs = [], [], [], []
    for k in range(n):
        r = Rotation.from_rotvec(rng.normal(size=3) * 0.5).as_matrix()
        vms.append(np.concatenate([r, rng.normal(size=(3, 1))], 1).astype(np.float32))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    vm_d = [dev(v) for v in vms]
    m_d = [torch.zeros(6, device="cuda") for _ in range(n)]
    v_d = [torch.zeros(6, device="cuda") for _ in range(n)]
    ref = [(v.astype(np.float64), np.zeros(6), np.zeros(6)) for v in vms]
    for t in range(1, 5):
        grads = [rng.normal(size=6) * 10.0 ** rng.integers(-3, 2) for _ in range(n)]
        g_d = [dev(g) for g in grads]
        items = [(vm_d[k], g_d[k], m_d[k], v_d[k], 1e-3, 2e-3, t) for k in range(n)]
        rtgs.pose_update(items)
        torch.cuda.synchronize()
        new_ref = []
        for k in range(n):
            # the oracle step starts from the kernel's float32 state
            vm0 = vm_prev[k] if t > 1 else vms[k].astype(np.float64)
            new_ref.append(oracle.pose_update(vm0, grads[k].astype(np.float32).astype(np.float64),
                                              m_prev[k] if t > 1 else np.zeros(6),
                                              v_prev[k] if t > 1 else np.zeros(6), t, 1e-3, 2e-3))
        vm_prev = [x.cpu().numpy().astype(np.float64) for x in vm_d]
        m_prev = [x.cpu().numpy().astype(np.float64) for x in m_d]
        v_prev = [x.cpu().numpy().astype(np.float64) for x in v_d]
        for k in range(n):
            np.testing.assert_allclose(vm_prev[k], new_ref[k][0], rtol=0, atol=2e-6)
            np.testing.assert_allclose(m_prev[k], new_ref[k][1], rtol=1e-6, atol=1e-30)
            np.testing.assert_allclose(v_prev[k], new_ref[k][2], rtol=1e-6, atol=1e-30)


def test_pose_update_rejects_bad_arguments():
    say("test_pose_update_rejects_bad_arguments")
    vm = torch.zeros(3, 4, device="cuda")
    z = torch.zeros(6, device="cuda")
    with pytest.raises(rtgs.RtgsError) as e:
        rtgs.pose_update([(vm, z, z.clone(), z.clone(), 1e-3, 1e-3, 0)])
    assert e.value.code == rtgs.RTGS_ERR_INVALID_ARG
