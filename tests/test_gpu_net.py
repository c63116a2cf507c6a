"""GPU learned force correction (libpm through its C ABI) against the FP64
oracle of the same network (net.c, pinned by finite differences).  The GPU
CNN takes BF16 activations and weights with FP32 accumulation, so parity is
by relative tolerance: forces <= 1e-2, loss <= 1e-2, gradients <= 2e-2
(relative L2 per parameter block)."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2007_13394_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def _params(seed, zero_out=False):
    rng = np.random.default_rng(seed)
    th = np.zeros(O.NET_NPARAM)
    for k, (o, n) in O.NET_OFF.items():
        fan = {"W0": 2, "W1": O.NET_H, "W2": O.NET_H, "W3": O.NET_H, "C1W": 27, "C2W": 27 * O.NET_C,
               "C3W": 27 * O.NET_C}.get(k, 1)
        s = (0.3 if k.startswith(("W", "B")) else 0.15) / np.sqrt(fan)
        th[o:o + n] = rng.standard_normal(n) * s
    if zero_out:
        for k in ("W3", "B3", "C3W", "C3B"):
            o, n = O.NET_OFF[k]
            th[o:o + n] = 0.0
    return th.astype(np.float32)


def _setup(name):
    from paper_2007_13394_amd import pm
    cfg = I.config(name)
    ctx = pm.Ctx(pm.make_config(cfg, flags=pm.PM_FLAG_LEARNED | pm.PM_FLAG_NO_SORT))
    return pm, cfg, ctx, O.make_sim(cfg)


def test_parameter_count_matches_the_oracle():
    from paper_2007_13394_amd import pm
    assert pm.pm_net_nparam() == O.NET_NPARAM


@pytest.mark.parametrize("name", ["C5_fd16", "C5_fd32"])
def test_zero_output_layers_give_the_plain_force(dev, name):
    pm, cfg, ctx, _ = _setup(name)
    x32, _ = I.synthetic_state(cfg, seed=31)
    x = torch.from_numpy(x32).to(dev)
    th = torch.from_numpy(_params(32, zero_out=True)).to(dev)
    acc = torch.empty_like(x)
    pm.pm_learned_force(ctx, th, 0.5, x, acc)
    ref = torch.empty_like(x)
    pm.pm_force(ctx, x, ref)
    e = rel_l2(acc.cpu().numpy(), ref.cpu().numpy())
    say(name, "learned (zero output layers) vs plain force rel L2", e)
    assert e < 1e-5


@pytest.mark.parametrize("name", ["C5_fd16", "C5_fd32"])
def test_learned_force_vs_oracle(dev, name):
    pm, cfg, ctx, sim = _setup(name)
    x32, _ = I.synthetic_state(cfg, seed=33)
    th32 = _params(34)
    x = torch.from_numpy(x32).to(dev)
    acc = torch.empty_like(x)
    pm.pm_learned_force(ctx, torch.from_numpy(th32).to(dev), 0.6, x, acc)
    ref = O.learned_force(sim, th32.astype(np.float64), 0.6, x32.astype(np.float64))
    plain = O.force_cont(sim, x32.astype(np.float64))
    e = rel_l2(acc.cpu().numpy(), ref)
    say(name, "learned force rel L2", e, "(correction vs plain:", rel_l2(ref, plain), ")")
    assert rel_l2(ref, plain) > 0.05     # the network does change the force
    assert e < 1e-2


@pytest.mark.parametrize("name", ["C5_fd16", "C5_fd32"])
def test_learned_loss_and_gradient_vs_oracle(dev, name):
    pm, cfg, ctx, sim = _setup(name)
    x32, _ = I.synthetic_state(cfg, seed=35)
    th32 = _params(36)
    rng = np.random.default_rng(37)
    target32 = (O.force_cont(sim, x32.astype(np.float64)) * (1 + 0.2 * rng.standard_normal(x32.shape))).astype(
        np.float32)
    x = torch.from_numpy(x32).to(dev)
    th = torch.from_numpy(th32).to(dev)
    d = torch.zeros_like(th)
    loss = pm.pm_learned_loss(ctx, th, 0.6, x, torch.from_numpy(target32).to(dev), d)
    rloss, rd = O.learned_loss(sim, th32.astype(np.float64), 0.6, x32.astype(np.float64),
                               target32.astype(np.float64))
    gd = d.cpu().numpy()
    say(name, "loss", loss, "oracle", rloss)
    assert abs(loss - rloss) / rloss < 1e-2
    for blk in (("W0", "B0", "W1", "B1", "W2", "B2", "W3", "B3"), ("C1W", "C1B"), ("C2W", "C2B"), ("C3W", "C3B")):
        idx = np.concatenate([np.arange(O.NET_OFF[k][0], O.NET_OFF[k][0] + O.NET_OFF[k][1]) for k in blk])
        e = rel_l2(gd[idx], rd[idx])
        say(name, "gradient block", blk[0], "rel L2", e)
        assert e < 2e-2


def test_adam_step_matches_definition(dev):
    from paper_2007_13394_amd import pm
    rng = np.random.default_rng(38)
    n = 1000
    th, m, v, g = (rng.standard_normal(n).astype(np.float32) for _ in range(4))
    v = np.abs(v)
    t = 3
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    T = [torch.from_numpy(a.copy()).to(dev) for a in (th, m, v, g)]
    pm.pm_adam(*T, lr, b1, b2, eps, t)
    m1 = b1 * m + (1 - b1) * g
    v1 = b2 * v + (1 - b2) * g * g
    th1 = th - lr * (m1 / (1 - b1 ** t)) / (np.sqrt(v1 / (1 - b2 ** t)) + eps)
    assert np.allclose(T[0].cpu().numpy(), th1, rtol=1e-5, atol=1e-6)


def test_learned_step_sorted_and_unsorted_agree(dev):
    """The tile-sorted learned step (particles come back permuted; ids map
    them back) against the unsorted one, and the unsorted one against kick
    and drift applied to the learned force."""
    from paper_2007_13394_amd import pm
    cfg = I.config("C1")
    n = cfg["n_mesh"]
    th = torch.from_numpy(_params(41)).to(dev)
    calls = [(0.5, 0.5, 0.55, 0.6), (0.6, 0.55, 0.65, 0.7)]
    x32, p32 = I.synthetic_state(cfg, seed=42)
    cs = pm.Ctx(pm.make_config(cfg, flags=pm.PM_FLAG_LEARNED))
    cu = pm.Ctx(pm.make_config(cfg, flags=pm.PM_FLAG_LEARNED | pm.PM_FLAG_NO_SORT))
    assert cs.sorts and not cu.sorts
    ids = torch.arange(cs.P, dtype=torch.int32, device=dev)
    pm.pm_attach_ids(cs, ids)
    xs, ps = torch.from_numpy(x32).to(dev), torch.from_numpy(p32).to(dev)
    xu, pu = xs.clone(), ps.clone()
    for i, c in enumerate(calls):
        if i == 0:
            acc = torch.empty_like(xu)
            pm.pm_learned_force(cu, th, c[0], xu, acc)
            kick, drift = pm.pm_kdk_factors(cu, *c)
            p_ref = pu.double() + kick * acc.double()
            x_ref = torch.remainder(xu.double() + drift * p_ref, n)
        pm.pm_learned_step(cs, th, xs, ps, *c)
        pm.pm_learned_step(cu, th, xu, pu, *c)
        if i == 0:
            ex = rel_l2(pu.cpu().numpy(), p_ref.cpu().numpy())
            dx = (xu.double() - x_ref).abs()
            dx = torch.minimum(dx, n - dx).max().item()
            say("unsorted learned step vs kick/drift of the learned force: p rel L2", ex, "max |dx|", dx)
            assert ex < 1e-6 and dx < 1e-4
    pm.pm_attach_ids(cs, None)
    order = torch.argsort(ids.long())
    xo, po = xs[:, order], ps[:, order]
    dx = (xo - xu).abs()
    dx = torch.minimum(dx, n - dx).max().item()
    ep = rel_l2(po.cpu().numpy(), pu.cpu().numpy())
    say("sorted vs unsorted learned steps: max |dx|", dx, "p rel L2", ep)
    assert dx < 1e-4 and ep < 1e-5


def test_learned_step_after_caller_moves_particles(dev):
    """A sorted learned step leaves the next step's tile counts; here the
    caller moves every particle in place before the second step, so the
    counts taken over are stale.  The sorted context must find that out after
    its scatter, redo the sort, the paint and the learned solve queued on the
    stale one, and agree with an unsorted context given the same moves."""
    from paper_2007_13394_amd import pm
    cfg = I.config("C1")
    n = cfg["n_mesh"]
    th = torch.from_numpy(_params(43)).to(dev)
    calls = [(0.5, 0.5, 0.55, 0.6), (0.6, 0.55, 0.65, 0.7)]
    x32, p32 = I.synthetic_state(cfg, seed=44)
    cs = pm.Ctx(pm.make_config(cfg, flags=pm.PM_FLAG_LEARNED))
    cu = pm.Ctx(pm.make_config(cfg, flags=pm.PM_FLAG_LEARNED | pm.PM_FLAG_NO_SORT))
    ids = torch.arange(cs.P, dtype=torch.int32, device=dev)
    pm.pm_attach_ids(cs, ids)
    xs, ps = torch.from_numpy(x32).to(dev), torch.from_numpy(p32).to(dev)
    xu, pu = xs.clone(), ps.clone()
    shift = torch.tensor([[5.5], [11.25], [2.0]], device=dev)
    for i, c in enumerate(calls):
        if i == 1:
            for xx in (xs, xu):   # same move on both, in place
                xx.add_(shift).remainder_(n)
                xx.masked_fill_(xx >= n, 0.0)
        pm.pm_learned_step(cs, th, xs, ps, *c)
        pm.pm_learned_step(cu, th, xu, pu, *c)
    pm.pm_attach_ids(cs, None)
    order = torch.argsort(ids.long())
    xo, po = xs[:, order], ps[:, order]
    dx = (xo - xu).abs()
    dx = torch.minimum(dx, n - dx).max().item()
    ep = rel_l2(po.cpu().numpy(), pu.cpu().numpy())
    say("learned steps with stale counts, sorted vs unsorted: max |dx|", dx, "p rel L2", ep)
    assert dx < 1e-4 and ep < 1e-5


def test_filter_table_and_its_vjp_vs_oracle(dev):
    from paper_2007_13394_amd import pm
    th32 = _params(51)
    th = torch.from_numpy(th32).to(dev)
    rng = np.random.default_rng(52)
    tbar = rng.standard_normal(O.NET_NB)
    for a in (0.05, 0.5, 1.0):
        tab = pm.pm_net_table(th, a).cpu().numpy()
        ref = O.net_table(th32.astype(np.float64), a)
        d = torch.zeros_like(th)
        pm.pm_net_table_vjp(th, a, torch.from_numpy(tbar).to(dev), d)
        dref = O.net_table_vjp(th32.astype(np.float64), a, tbar)
        e_t, e_d = np.max(np.abs(tab - ref)), rel_l2(d.cpu().numpy(), dref)
        say("a", a, "table max abs err", e_t, "vjp rel L2", e_d)
        assert e_t < 1e-5 and e_d < 1e-4


def _golden_256():
    import importlib.util
    import json
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("make_learned_force", os.path.join(here, "make_learned_force.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    with open(os.path.join(here, "learned_force_256.json")) as f:
        return mod, json.load(f)


def test_learned_force_two_pass_transforms_vs_oracle_256(dev):
    """On meshes of 256^3 and more the learned force runs on the two-pass
    transforms: the density and the CNN output each through rows with the
    first axis-0 digit and axis 1, one pass B that forms the potential's
    gradient factor from both (radial filter on the density part), and the
    plain solve's inverse passes.  Against the FP64 oracle's learned force at
    4096 sampled particles (fixture of tests/golden/make_learned_force.py):
    the force within 1e-2 and its correction over the plain force within
    3e-2 (relative L2).  The sorted learned step (float32 density from the
    tile paint) must then match the unsorted one."""
    from paper_2007_13394_amd import pm
    mod, ref = _golden_256()
    cfg = I.config(ref["config"]["name"], n_cdm=ref["config"]["n_cdm"], n_sites=ref["config"]["n_sites"])
    assert cfg["n_mesh"] == 256
    n = cfg["n_mesh"]
    th32 = mod.params(ref["theta_seed"])
    th = torch.from_numpy(th32).to(dev)
    x32, p32 = I.synthetic_state(cfg, seed=ref["state_seed"])
    idx = np.array(ref["index"])
    cu = pm.Ctx(pm.make_config(cfg, flags=pm.PM_FLAG_LEARNED | pm.PM_FLAG_NO_SORT))
    xu = torch.from_numpy(x32).to(dev)
    acc = torch.empty_like(xu)
    pm.pm_learned_force(cu, th, ref["a"], xu, acc)
    got = acc.cpu().numpy().astype(np.float64)[:, idx]
    want, plain = np.array(ref["force"]), np.array(ref["plain_force"])
    e_f = rel_l2(got, want)
    e_c = rel_l2(got - plain, want - plain)
    say("learned force at 256^3 (two-pass transforms) vs oracle: rel L2", e_f, "; correction", e_c,
        "; correction / plain force", rel_l2(want, plain))
    assert e_f < 1e-2 and e_c < 3e-2
    # sorted (float32 density, fused counts) against unsorted learned steps
    cs = pm.Ctx(pm.make_config(cfg, flags=pm.PM_FLAG_LEARNED))
    ids = torch.arange(cs.P, dtype=torch.int32, device=dev)
    pm.pm_attach_ids(cs, ids)
    xs, ps = torch.from_numpy(x32).to(dev), torch.from_numpy(p32).to(dev)
    xu, pu = xs.clone(), ps.clone()
    for c in [(0.5, 0.5, 0.55, 0.6), (0.6, 0.55, 0.65, 0.7)]:
        pm.pm_learned_step(cs, th, xs, ps, *c)
        pm.pm_learned_step(cu, th, xu, pu, *c)
    pm.pm_attach_ids(cs, None)
    order = torch.argsort(ids.long())
    xo, po = xs[:, order], ps[:, order]
    dx = (xo - xu).abs()
    dx = torch.minimum(dx, n - dx).max().item()
    ep = rel_l2(po.cpu().numpy(), pu.cpu().numpy())
    say("256^3 sorted vs unsorted learned steps: max |dx|", dx, "p rel L2", ep)
    assert dx < 1e-3 and ep < 1e-5
