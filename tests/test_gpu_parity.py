"""GPU path (libpm through its C ABI) against the FP64 oracle on identical
seeded inputs.  Bars: bit-exact int64 paint; relative L2 <= 1e-5 for forces,
momenta and displacements of one step (FP32 state); FFT relative L2 <= 1e-6."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2007_13394_amd import inputs as I

pytestmark = pytest.mark.gpu


def _pm():
    from paper_2007_13394_amd import pm
    return pm


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    t = np.complex128 if (np.iscomplexobj(a) or np.iscomplexobj(b)) else np.float64
    a, b = a.astype(t), b.astype(t)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def min_image(d, n):
    return (d + n / 2) % n - n / 2


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def c1():
    pm = _pm()
    cfg = I.config("C1")
    ctx = pm.Ctx(pm.make_config(cfg))
    return cfg, ctx


def test_segments_and_shells_match_oracle(c1):
    pm = _pm()
    cfg, ctx = c1
    off, mass, q = pm.pm_segments(ctx)
    s = O.make_sim(cfg)
    o_off, o_mass, o_q = O.segments(s)
    assert np.array_equal(off, o_off)
    assert np.allclose(mass, o_mass, rtol=1e-11, atol=0)
    assert np.all(np.abs(q - o_q) <= 1)
    e, qs, ms = pm.pm_shells(ctx)
    oe, oq, om = O.fd_shells([1.0, 1.0, 1.0], 10)
    assert np.allclose(e, oe, rtol=1e-10, atol=1e-12) and np.allclose(qs, oq, rtol=1e-10)
    assert np.allclose(ms, om, rtol=1e-10)
    a = np.array([0.01, 0.05, 0.3, 1.0])
    D, G = pm.pm_growth(ctx, a)
    oD, oG = O.growth(s.cosmo, a)
    assert np.allclose(D, oD, rtol=1e-8) and np.allclose(G, oG, rtol=1e-8)


def test_shells_normal_hierarchy_match_oracle():
    # the effective distribution of three unequal masses (cut-off q = 30 / alpha_min)
    pm = _pm()
    cfg = I.config("C1", m_nu=I.NH_006)
    ctx = pm.Ctx(pm.make_config(cfg))
    e, qs, ms = pm.pm_shells(ctx)
    alpha = np.array(I.NH_006) / I.NH_006[0]
    oe, oq, om = O.fd_shells(alpha, 10)
    assert np.allclose(e, oe, rtol=1e-9) and np.allclose(qs, oq, rtol=1e-9) and np.allclose(ms, om, rtol=1e-9)
    off, mass, q = pm.pm_segments(ctx)
    _, o_mass, _ = O.segments(O.make_sim(cfg))
    assert np.allclose(mass, o_mass, rtol=1e-9)


def test_paint_bit_exact_synthetic_and_adversarial(c1, dev):
    pm = _pm()
    cfg, ctx = c1
    n = cfg["n_mesh"]
    x, _ = I.synthetic_state(cfg, seed=5)
    adv = I.adversarial_positions(n, 4000, seed=6)
    Qm = 3 * 2 ** 40 + 12345
    for arr in (x, adv):
        say("paint", arr.shape)
        xd = torch.from_numpy(arr).to(dev)
        mesh = torch.zeros(n ** 3, dtype=torch.int64, device=dev)
        pm.pm_paint_q(ctx, xd, 0, arr.shape[1], Qm, mesh)
        got = mesh.cpu().numpy().reshape(n, n, n)
        ref = O.paint_q(arr.astype(np.float64), 0, arr.shape[1], Qm, n)
        assert np.array_equal(got, ref)
        assert got.sum() == arr.shape[1] * Qm


def test_paint_segments_and_order_independence(c1, dev):
    pm = _pm()
    cfg, ctx = c1
    n = cfg["n_mesh"]
    x, _ = I.synthetic_state(cfg, seed=7)
    xd = torch.from_numpy(x).to(dev)
    mesh = torch.zeros(n ** 3, dtype=torch.int64, device=dev)
    pm.pm_paint(ctx, xd, 0, ctx.nseg, mesh)
    got = mesh.cpu().numpy().reshape(n, n, n)
    off, _, q = pm.pm_segments(ctx)
    s = O.make_sim(cfg)
    o_off, _, o_q = O.segments(s)
    assert np.array_equal(off, o_off) and np.all(np.abs(q - o_q) <= 1)
    # the oracle paints each segment with the library's quantum: identical integers
    ref = np.zeros((n, n, n), dtype=np.int64)
    for g in range(len(q)):
        O.paint_q(x.astype(np.float64), int(off[g]), int(off[g + 1] - off[g]), int(q[g]), n, ref)
    assert np.array_equal(got, ref)
    # shuffle within each segment: identical mesh
    rng = np.random.default_rng(1)
    xs = x.copy()
    for g in range(len(off) - 1):
        perm = rng.permutation(np.arange(off[g], off[g + 1]))
        xs[:, off[g]:off[g + 1]] = x[:, perm]
    mesh2 = torch.zeros_like(mesh)
    pm.pm_paint(ctx, torch.from_numpy(xs).to(dev), 0, ctx.nseg, mesh2)
    assert torch.equal(mesh, mesh2)


@pytest.mark.parametrize("n", [16, 64, 128, 256, 512])
def test_fft_r2c_and_c2r_vs_oracle(dev, n):
    pm = _pm()
    cfg = I.config("C1", n_mesh=n, n_cdm=16, n_sites=2)
    ctx = pm.Ctx(pm.make_config(cfg))
    r = np.random.default_rng(n).normal(size=(n, n, n)).astype(np.float32)
    out = torch.empty(n * n * (n // 2 + 1), dtype=torch.complex64, device=dev)
    pm.pm_fft_r2c(ctx, torch.from_numpy(r).to(dev), out)
    got = out.cpu().numpy().reshape(n, n, n // 2 + 1)
    ref = O.rfft3d(r.astype(np.float64))
    say("fft", n, rel_l2(got, ref))
    assert rel_l2(got, ref) < 1e-6
    back = torch.empty(n ** 3, dtype=torch.float32, device=dev)
    pm.pm_fft_c2r(ctx, torch.from_numpy(ref.astype(np.complex64)).to(dev), back)
    refb = O.irfft3d(ref)
    assert rel_l2(back.cpu().numpy().reshape(n, n, n), refb) < 1e-6


@pytest.mark.parametrize("n", [64, 256])
def test_force_mesh_vs_oracle(dev, n):
    pm = _pm()
    cfg = I.config("C1", n_mesh=n, n_cdm=32, n_sites=8)
    ctx = pm.Ctx(pm.make_config(cfg))
    q = I.synthetic_density_q(n, seed=9)
    out = torch.empty(3 * n ** 3, dtype=torch.float32, device=dev)
    pm.pm_force_mesh(ctx, torch.from_numpy(q).to(dev), out)
    got = out.cpu().numpy().reshape(3, n, n, n)
    ref = O.force_mesh(q, 40, cfg["omega_m"])
    for d in range(3):
        say("force mesh", d, rel_l2(got[d], ref[d]))
        assert rel_l2(got[d], ref[d]) < 1e-5


def test_force_on_particles_vs_oracle(c1, dev):
    pm = _pm()
    cfg, ctx = c1
    x, _ = I.synthetic_state(cfg, seed=11)
    acc = torch.empty_like(torch.from_numpy(x)).to(dev)
    pm.pm_force(ctx, torch.from_numpy(x).to(dev), acc)
    got = acc.cpu().numpy()
    ref = O.force(O.make_sim(cfg), x.astype(np.float64))
    nc = cfg["n_cdm"] ** 3
    say("force", rel_l2(got, ref), rel_l2(got[:, :nc], ref[:, :nc]), rel_l2(got[:, nc:], ref[:, nc:]))
    assert rel_l2(got, ref) < 1e-5
    assert rel_l2(got[:, :nc], ref[:, :nc]) < 1e-5 and rel_l2(got[:, nc:], ref[:, nc:]) < 1e-5


CALLS = [(0.01, 0.01, 0.0595, 0.109), (0.604, 0.5545, 0.6535, 0.703), (1.0, 0.9505, 1.0, 1.0)]


def _step_compare(cfg, gx, gp, x, p, call):
    n = cfg["n_mesh"]
    s = O.make_sim(cfg)
    kick, drift = O.kdk_factors(s.cosmo, *[[v] for v in call])
    ox, op = x.astype(np.float64), p.astype(np.float64)
    O.step(s, ox, op, kick[0], drift[0])
    ox32, op32 = ox.astype(np.float32), op.astype(np.float32)
    nc = cfg["n_cdm"] ** 3
    dp_g, dp_o = gp.astype(np.float64) - p, op32.astype(np.float64) - p
    dx_g = min_image(gx.astype(np.float64) - x, n)
    dx_o = min_image(ox32.astype(np.float64) - x, n)
    for sl in (slice(0, nc), slice(nc, None)):
        if dp_g[:, sl].size == 0:
            continue
        say("step", call, rel_l2(dp_g[:, sl], dp_o[:, sl]), rel_l2(dx_g[:, sl], dx_o[:, sl]) if drift[0] else 0)
        assert rel_l2(dp_g[:, sl], dp_o[:, sl]) < 1e-5
        if drift[0] != 0:
            assert rel_l2(dx_g[:, sl], dx_o[:, sl]) < 1e-5
        else:
            assert np.array_equal(gx[:, sl], x[:, sl])
    assert np.all((gx >= 0) & (gx < n))


@pytest.mark.parametrize("call", CALLS)
def test_one_step_sorted_vs_oracle(c1, dev, call):
    """Default step: particles are tile-sorted; ids map them back."""
    pm = _pm()
    cfg, ctx = c1
    x, p = I.synthetic_state(cfg, seed=13)
    pm.pm_reset_order(ctx)
    ids = torch.arange(ctx.P, dtype=torch.int32, device=dev)
    pm.pm_attach_ids(ctx, ids)
    xd, pd = torch.from_numpy(x).to(dev), torch.from_numpy(p).to(dev)
    pm.pm_step(ctx, xd, pd, *call)
    order = np.argsort(ids.cpu().numpy())
    assert np.array_equal(np.sort(ids.cpu().numpy()), np.arange(ctx.P))
    gx, gp = xd.cpu().numpy()[:, order], pd.cpu().numpy()[:, order]
    tags = pm.pm_segment_tags(ctx).cpu().numpy()[order]
    off, _, _ = pm.pm_segments(ctx)
    assert np.array_equal(tags, np.repeat(np.arange(ctx.nseg), np.diff(off)))
    pm.pm_attach_ids(ctx, None)
    pm.pm_reset_order(ctx)
    _step_compare(cfg, gx, gp, x, p, call)


@pytest.mark.parametrize("call", CALLS[:2])
def test_one_step_unsorted_vs_oracle(dev, call):
    pm = _pm()
    cfg = I.config("C1")
    ctx = pm.Ctx(pm.make_config(cfg, flags=pm.PM_FLAG_NO_SORT))
    x, p = I.synthetic_state(cfg, seed=13)
    xd, pd = torch.from_numpy(x).to(dev), torch.from_numpy(p).to(dev)
    pm.pm_step(ctx, xd, pd, *call)
    _step_compare(cfg, xd.cpu().numpy(), pd.cpu().numpy(), x, p, call)


def test_sorted_state_paint_and_force_are_order_independent(dev):
    # after sorted steps the particle arrays are permuted; painting and forces
    # through the segment tags must match the same particles in canonical order
    pm = _pm()
    cfg = I.config("C1")
    ctx = pm.Ctx(pm.make_config(cfg))
    n = cfg["n_mesh"]
    x, p = I.synthetic_state(cfg, seed=31)
    ids = torch.arange(ctx.P, dtype=torch.int32, device=dev)
    pm.pm_attach_ids(ctx, ids)
    xd, pd = torch.from_numpy(x).to(dev), torch.from_numpy(p).to(dev)
    for c in CALLS[:2]:
        pm.pm_step(ctx, xd, pd, *c)
    order = torch.argsort(ids.long())
    xc = xd[:, order].contiguous()
    m_perm = torch.zeros(n ** 3, dtype=torch.int64, device=dev)
    pm.pm_paint(ctx, xd, 0, ctx.nseg, m_perm)
    m_nu = torch.zeros_like(m_perm)
    pm.pm_paint(ctx, xd, 1, ctx.nseg, m_nu)
    acc_perm = torch.empty_like(xd)
    pm.pm_force(ctx, xd, acc_perm)
    k1, pk1, _ = pm.pm_power(ctx, xd, 0, 1, 1, ctx.nseg, nbins=16)
    ctx2 = pm.Ctx(pm.make_config(cfg, flags=pm.PM_FLAG_NO_SORT))
    m_can = torch.zeros_like(m_perm)
    pm.pm_paint(ctx2, xc, 0, ctx2.nseg, m_can)
    m_nu2 = torch.zeros_like(m_perm)
    pm.pm_paint(ctx2, xc, 1, ctx2.nseg, m_nu2)
    assert torch.equal(m_perm, m_can) and torch.equal(m_nu, m_nu2)
    acc_can = torch.empty_like(xc)
    pm.pm_force(ctx2, xc, acc_can)
    assert torch.allclose(acc_perm[:, order], acc_can, rtol=0, atol=1e-6 * float(acc_can.abs().max()))
    k2, pk2, _ = pm.pm_power(ctx2, xc, 0, 1, 1, ctx2.nseg, nbins=16)
    assert np.allclose(pk1, pk2, rtol=1e-5, atol=0)


def test_initial_conditions_vs_oracle(c1, dev):
    # The momentum is (G/D)(a0) times the displacement field, so it carries
    # the displacement at full float32 precision; positions are float32 values
    # of q + s and are compared to the oracle's rounded position within an ulp.
    pm = _pm()
    cfg, ctx = c1
    n = cfg["n_mesh"]
    w = I.white_noise(21, cfg["n_cdm"])
    x, p = ctx.particles()
    pm.pm_ic(ctx, torch.from_numpy(w).to(dev), x, p)
    gx, gp = x.cpu().numpy(), p.cpu().numpy().astype(np.float64)
    ox, op = O.ic(O.make_sim(cfg), w)
    nc = cfg["n_cdm"] ** 3
    ulp = np.spacing(np.float32(n))
    dx = np.abs(min_image(gx.astype(np.float64) - ox.astype(np.float32).astype(np.float64), n))
    say("ic", rel_l2(gp[:, :nc], op[:, :nc]), rel_l2(gp[:, nc:], op[:, nc:]), dx.max() / ulp)
    assert rel_l2(gp[:, :nc], op[:, :nc]) < 1e-5
    assert rel_l2(gp[:, nc:], op[:, nc:]) < 1e-5
    assert dx[:, :nc].max() <= ulp and dx[:, nc:].max() <= 2 * ulp
    assert np.all((gx >= 0) & (gx < n))


def test_power_spectrum_vs_oracle(c1, dev):
    pm = _pm()
    cfg, ctx = c1
    x, _ = I.synthetic_state(cfg, seed=17)
    xd = torch.from_numpy(x).to(dev)
    s = O.make_sim(cfg)
    nseg = ctx.nseg
    dm = O.delta_of(s, x.astype(np.float64), 0, nseg)
    dc = O.delta_of(s, x.astype(np.float64), 0, 1)
    dn = O.delta_of(s, x.astype(np.float64), 1, nseg)
    for (alo, ahi, blo, bhi), da, db in (((0, nseg, 0, nseg), dm, None), ((0, 1, 1, nseg), dc, dn)):
        for comp in (False, True):
            k, pk, nm = pm.pm_power(ctx, xd, alo, ahi, blo, bhi, nbins=32, compensate=comp)
            ok, opk, onm = O.power(da, db, cfg["box"], 32, comp)
            assert np.array_equal(nm, onm)
            assert np.allclose(k, ok, rtol=1e-12)
            sel = onm > 0
            err = np.abs(pk[sel] - opk[sel]) / np.abs(opk[sel]).max()
            say("power", alo, ahi, blo, bhi, comp, err.max())
            assert err.max() < 1e-5


def test_one_step_C5_vs_oracle(dev):
    # 256^3 mesh: column and axis-0 passes on the register six-step transform
    pm = _pm()
    cfg = I.config("C5")
    ctx = pm.Ctx(pm.make_config(cfg))
    x, p = I.synthetic_state(cfg, seed=41)
    ids = torch.arange(ctx.P, dtype=torch.int32, device=dev)
    pm.pm_attach_ids(ctx, ids)
    xd, pd = torch.from_numpy(x).to(dev), torch.from_numpy(p).to(dev)
    call = (0.406, 0.3565, 0.4555, 0.505)
    pm.pm_step(ctx, xd, pd, *call)
    order = np.argsort(ids.cpu().numpy())
    _step_compare(cfg, xd.cpu().numpy()[:, order], pd.cpu().numpy()[:, order], x, p, call)


@pytest.mark.parametrize("variant", ["massless", "nfib20"])
def test_one_step_runtime_increase_configs_vs_oracle(dev, variant):
    """The two configurations the runtime-increase experiment (Table 1, Sec. 4)
    times besides the default: no neutrino particles (one segment, CDM only,
    massless background) and N_fib = 20 (41 directions, 410 particles per
    site), one sorted step each against the oracle."""
    pm = _pm()
    if variant == "massless":
        cfg = I.config("C5", n_sites=0, m_nu=(0.0, 0.0, 0.0))
    else:
        cfg = I.config("C1", n_fib=20)
    ctx = pm.Ctx(pm.make_config(cfg))
    assert ctx.sorts
    assert ctx.nseg == (1 if variant == "massless" else 11)
    x, p = I.synthetic_state(cfg, seed=43)
    ids = torch.arange(ctx.P, dtype=torch.int32, device=dev)
    pm.pm_attach_ids(ctx, ids)
    xd, pd = torch.from_numpy(x).to(dev), torch.from_numpy(p).to(dev)
    call = CALLS[1]
    pm.pm_step(ctx, xd, pd, *call)
    pm.pm_attach_ids(ctx, None)
    order = np.argsort(ids.cpu().numpy())
    _step_compare(cfg, xd.cpu().numpy()[:, order], pd.cpu().numpy()[:, order], x, p, call)


def test_device_guards_report_overflow_and_nan(dev):
    """The end-of-call guards: a one-cell clump whose int64 sum passes 2^63
    (shift 52, 300 CDM particles on one lattice point, integer arithmetic
    only) returns PM_ERR_OVERFLOW from pm_force; a non-finite momentum
    returns PM_ERR_NAN from pm_step.  Both are flags the kernels raise; the
    state stays in bounds."""
    pm = _pm()
    cfg = I.config("C1", shift=52)
    ctx = pm.Ctx(pm.make_config(cfg, flags=pm.PM_FLAG_NO_SORT))
    off, _, q = pm.pm_segments(ctx)
    assert 2 ** 63 // int(q[0]) < 300 < 2 ** 64 // int(q[0])
    x, p = I.synthetic_state(cfg, seed=51)
    x[:, :300] = np.float32(10.0)
    xd, pd = torch.from_numpy(x).to(dev), torch.from_numpy(p).to(dev)
    acc = torch.empty_like(xd)
    with pytest.raises(pm.PMError) as e:
        pm.pm_force(ctx, xd, acc)
    assert e.value.status == pm.PM_ERR_OVERFLOW
    # below the limit the same clump is fine
    x[:, :300] = x[:, 300:600]
    x[:, :150] = np.float32(10.0)
    pm.pm_force(ctx, torch.from_numpy(x).to(dev), acc)
    ctx2 = pm.Ctx(pm.make_config(I.config("C1")))
    x2, p2 = I.synthetic_state(I.config("C1"), seed=52)
    p2[1, 1234] = np.nan
    with pytest.raises(pm.PMError) as e:
        pm.pm_step(ctx2, torch.from_numpy(x2).to(dev), torch.from_numpy(p2).to(dev), *CALLS[1])
    assert e.value.status == pm.PM_ERR_NAN


def test_deferred_guards(dev):
    """PM_FLAG_DEFER_GUARDS: sorted steps give the same particles bit for bit
    as with the default check; a step that makes a momentum non-finite
    returns PM_OK and the next guarded call reports PM_ERR_NAN; pm_sync
    reports a failure of the last call, and nothing once it is consumed."""
    pm = _pm()
    cfg = I.config("C1")
    x, p = I.synthetic_state(cfg, seed=53)
    runs = []
    for flags in (0, pm.PM_FLAG_DEFER_GUARDS):
        ctx = pm.Ctx(pm.make_config(cfg, flags=flags))
        ids = torch.arange(ctx.P, dtype=torch.int32, device=dev)
        pm.pm_attach_ids(ctx, ids)   # the order within a tile key varies run to run
        xd, pd = torch.from_numpy(x).to(dev), torch.from_numpy(p).to(dev)
        for c in CALLS:
            pm.pm_step(ctx, xd, pd, *c)
        pm.pm_sync(ctx)
        pm.pm_attach_ids(ctx, None)
        order = torch.argsort(ids.long())
        runs.append((xd[:, order].cpu(), pd[:, order].cpu()))
    assert torch.equal(runs[0][0], runs[1][0]) and torch.equal(runs[0][1], runs[1][1])
    # every step starts from finite positions (one momentum is NaN), as in
    # the guard test above; states that came out non-finite are not stepped
    ctx = pm.Ctx(pm.make_config(cfg, flags=pm.PM_FLAG_DEFER_GUARDS))
    pn = p.copy()
    pn[1, 1234] = np.nan

    def state(mom):
        pm.pm_reset_order(ctx)                  # a fresh state is in canonical order
        return torch.from_numpy(x).to(dev), torch.from_numpy(mom).to(dev)

    pm.pm_step(ctx, *state(pn), *CALLS[0])      # the failing call itself returns PM_OK
    with pytest.raises(pm.PMError) as e:
        pm.pm_step(ctx, *state(p), *CALLS[0])   # ... and the next guarded call reports it
    assert e.value.status == pm.PM_ERR_NAN
    pm.pm_sync(ctx)                             # that finite step's own check is clean
    pm.pm_step(ctx, *state(pn), *CALLS[1])      # non-finite again, now reported by pm_sync
    with pytest.raises(pm.PMError) as e:
        pm.pm_sync(ctx)
    assert e.value.status == pm.PM_ERR_NAN
    pm.pm_sync(ctx)                             # consumed: nothing pending


def test_sorted_step_after_caller_moves_particles(dev):
    """A sorted step leaves the tile counts of the positions it wrote for the
    next step's sort, which checks them after its scatter.  Here the caller
    moves every particle between two steps (same array): the check must
    reject the stale counts and the step must still match the oracle."""
    pm = _pm()
    cfg = I.config("C1")
    n = cfg["n_mesh"]
    ctx = pm.Ctx(pm.make_config(cfg))
    x, p = I.synthetic_state(cfg, seed=71)
    ids = torch.arange(ctx.P, dtype=torch.int32, device=dev)
    pm.pm_attach_ids(ctx, ids)
    xd, pd = torch.from_numpy(x).to(dev), torch.from_numpy(p).to(dev)
    pm.pm_step(ctx, xd, pd, *CALLS[0])
    # move the particles in place: the counts the step left no longer match
    xd.add_(torch.tensor([[7.25], [19.5], [3.0]], device=dev)).remainder_(n)
    xd.masked_fill_(xd >= n, 0.0)
    order = np.argsort(ids.cpu().numpy())
    x1, p1 = np.ascontiguousarray(xd.cpu().numpy()[:, order]), np.ascontiguousarray(pd.cpu().numpy()[:, order])
    pm.pm_step(ctx, xd, pd, *CALLS[1])
    pm.pm_attach_ids(ctx, None)
    order = np.argsort(ids.cpu().numpy())
    _step_compare(cfg, xd.cpu().numpy()[:, order], pd.cpu().numpy()[:, order], x1, p1, CALLS[1])


def test_sorted_steps_with_a_clump_and_fast_streamers_vs_oracle(dev):
    """Two sorted steps (the second takes over the tile counts the first
    readout wrote) on a state with a quarter of the CDM in one clump of 2^3
    cells, so one tile holds thousands of particles and its paint and
    readout loop over many rounds, and with every neutrino moving about 40
    cells (2.5 tiles) per step in a random direction, so the next-step key
    counts of the readout fall outside its 27-tile histogram.  Each step
    matches the oracle's step from the same state."""
    pm = _pm()
    cfg = I.config("C1")
    n = cfg["n_mesh"]
    ctx = pm.Ctx(pm.make_config(cfg))
    assert ctx.sorts
    x, p = I.synthetic_state(cfg, seed=81)
    rng = np.random.default_rng(82)
    nc = cfg["n_cdm"] ** 3
    m = nc // 4
    x[:, :m] = (np.float32(30.0) + rng.uniform(0.0, 2.0, size=(3, m))).astype(np.float32)
    s = O.make_sim(cfg)
    calls = CALLS[1:]
    _, drift = O.kdk_factors(s.cosmo, *[[v] for v in calls[0]])
    dirs = rng.standard_normal((3, ctx.P - nc))
    dirs /= np.linalg.norm(dirs, axis=0)
    p[:, nc:] = (40.0 / drift[0] * dirs).astype(np.float32)
    ids = torch.arange(ctx.P, dtype=torch.int32, device=dev)
    pm.pm_attach_ids(ctx, ids)
    xd, pd = torch.from_numpy(np.ascontiguousarray(x)).to(dev), torch.from_numpy(np.ascontiguousarray(p)).to(dev)
    xs, ps = x, p
    for call in calls:
        pm.pm_step(ctx, xd, pd, *call)
        order = np.argsort(ids.cpu().numpy())
        gx, gp = xd.cpu().numpy()[:, order], pd.cpu().numpy()[:, order]
        _step_compare(cfg, gx, gp, xs, ps, call)
        xs, ps = np.ascontiguousarray(gx), np.ascontiguousarray(gp)
    pm.pm_attach_ids(ctx, None)
