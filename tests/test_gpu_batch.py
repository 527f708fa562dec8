"""Batched instances: one stage launch covers every instance's tiles.

Checks per-instance parity with the oracle, bitwise equality with separate
single-instance runs, HIP-graph replays against eager launches (several
replays with eager work and synchronisation in between), and the autotuner.
"""
import json
import os

import numpy as np
import pytest

import olb_inputs as I
import oracle
from _metrics import moment_errors, rel_scalar

pytestmark = pytest.mark.gpu

TOL64 = 1e-11


def _olb():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_1702_01690_amd import olb
    return olb


def _channels(precision=0):
    cases = [I.channel(70, 20, tw=0.75 * I.T_CRIT, seed=11),
             I.channel(40, 33, tw=0.90 * I.T_CRIT, seed=12),
             I.channel(129, 12, tw=0.80 * I.T_CRIT, seed=13)]
    for c in cases:
        c.params["precision"] = precision
        c.params["rho_ref"] = I.N_CRIT
    return cases


def _periodic():
    a = I.shear32()
    b = I.spinodal(66, 45, seed=21)
    b.params["ds"] = a.params["ds"]     # instances may differ in every parameter
    return [a, b]


def _oracle_run(case, steps):
    o = oracle.Oracle(case.params)
    o.set_fields(*case.fields)
    o.step(steps)
    return o.moments()


def _batch(cases, graph=0, by=None):
    olb = _olb()
    b = olb.Batch([c.params for c in cases])
    if by:
        b.set_tile(by)
    if graph:
        b.use_graph(graph)
    for i, c in enumerate(cases):
        b.set_fields(i, *c.fields)
    return b


@pytest.mark.parametrize("kind", ["walls", "periodic"])
def test_batch_fp64_matches_oracle_per_instance(kind):
    cases = _channels() if kind == "walls" else _periodic()
    steps = 20
    print(f"[batch] {kind}: {[c.name for c in cases]} steps={steps}", flush=True)
    b = _batch(cases)
    b.step(steps)
    b.sync()
    for i, c in enumerate(cases):
        err = moment_errors(b.moments(i), _oracle_run(c, steps))
        print(f"[batch] {c.name}: {err}", flush=True)
        assert max(err.values()) < TOL64, (c.name, err)


def test_batch_half_channels_match_oracle_per_instance():
    cases = [I.half_channel(70, 20, seed=31, tw=0.75 * I.T_CRIT), I.half_channel(9, 33, seed=32),
             I.half_channel(130, 7, seed=33, tw=0.9 * I.T_CRIT, uw=0.02)]
    steps = 15
    b = _batch(cases)
    b.step(steps)
    b.sync()
    for i, c in enumerate(cases):
        err = moment_errors(b.moments(i), _oracle_run(c, steps))
        print(f"[batch] {c.name}: {err}", flush=True)
        assert max(err.values()) < TOL64, (c.name, err)


def test_batch_equals_single_instance_runs_bitwise():
    olb = _olb()
    cases = _channels()
    b = _batch(cases)
    b.step(7)
    for i, c in enumerate(cases):
        lat = olb.Lattice(c.params)
        lat.set_fields(*c.fields)
        lat.step(7)
        np.testing.assert_array_equal(b.get_f(i), lat.get_f())
        lo, hi = lat.wall_density()
        blo, bhi = b.wall_density(i)
        np.testing.assert_array_equal(blo, lo)
        np.testing.assert_array_equal(bhi, hi)


def test_batch_mixing_storage_orders_equals_single_runs_bitwise():
    """A batch whose instances use different storage orders: the 66 x 45
    lattice interleaves the rows of its populations, the 4096 x 2624 FP64
    lattice (25 x 2630 x 4096 x 8 B > 2^31) keeps one plane per population.
    One launch per stage covers both; each instance's moments equal those of
    its own single-instance run, bitwise."""
    olb = _olb()
    small = I.spinodal(66, 45, seed=21)
    big = I.spinodal(64, 64, seed=22)
    nx, ny = 4096, 2624
    big.params.update(nx=nx, ny=ny)
    big = I.Case("spinodal4096x2624tiled", big.params,
                 *(np.tile(a, (ny // 64, nx // 64)) for a in big.fields), 0)
    assert 25 * (ny + 6) * nx * 8 > 2 ** 31 > 25 * (45 + 6) * 66 * 8
    cases = [small, big]
    print("[batch] interleaved 66x45 + planes 4096x2624, FP64, 5 steps", flush=True)
    b = _batch(cases)
    b.step(5)
    b.sync()
    for i, c in enumerate(cases):
        lat = olb.Lattice(c.params)
        lat.set_fields(*c.fields)
        lat.step(5)
        for x, y in zip(b.moments(i), lat.moments()):
            np.testing.assert_array_equal(x, y)
        del lat


@pytest.mark.parametrize("by", [8, 16])
def test_graph_replays_match_eager_launches(by):
    cases = _channels()
    g = _batch(cases, graph=2, by=by)
    e = _batch(cases, by=by)
    for rnd, steps in enumerate((4, 3, 6)):
        g.step(steps)          # graph replays (+ one direct step when odd)
        e.step(steps)
        g.sync()
        e.sync()
        for i in range(len(cases)):
            # eager work between replays: read-outs through other kernels
            gm, em = g.moments(i), e.moments(i)
            for a, bb in zip(gm, em):
                np.testing.assert_array_equal(a, bb)
        print(f"[batch] graph round {rnd} ({steps} steps) bitwise equal", flush=True)
    np.testing.assert_array_equal(g.get_f(1), e.get_f(1))


def test_batch_tile_order_does_not_change_results():
    cases = _channels()
    a = _batch(cases)
    b = _batch(cases)
    b.set_tile_order(2)
    a.step(5)
    b.step(5)
    for i in range(len(cases)):
        np.testing.assert_array_equal(a.get_f(i), b.get_f(i))


@pytest.mark.parametrize("precision,graph", [(0, 0), (1, 2)])
def test_autotune_picks_a_launch_configuration_and_caches_it(tmp_path, precision, graph):
    """The autotuner's search (tile height, tile order, steps per graph) picks
    a valid configuration, caches it, reads it back for a batch of the same
    shape, and leaves the results bitwise those of the default
    configuration."""
    olb = _olb()
    cases = _channels(precision=precision)
    cache = str(tmp_path / "tune.json")
    b = olb.Batch([c.params for c in cases])
    if graph:
        b.use_graph(graph)
    by = b.autotune(trial_steps=2, cache_path=cache)
    cfg = b.launch_config()
    print(f"[batch] autotune precision={precision} graph={graph}: {cfg}", flush=True)
    assert by == cfg[0] and by in ((8, 12, 16) if precision else (8, 16))
    assert cfg[1] in (0, 4, 8, 16)
    assert cfg[2] == 0 if not graph else cfg[2] in (2, 10, 30)
    data = json.load(open(cache))
    entry = next(iter(data.values()))
    assert (entry["by"], entry["strip"], entry["graph"]) == cfg and len(entry["ms_per_step"]) >= 6
    # the trial discarded the state: stepping now is an error
    with pytest.raises(olb.OlbError) as e:
        b.step(1)
    assert e.value.code == olb.OLB_E_STATE
    # a second batch of the same shape reads the cache
    b2 = olb.Batch([c.params for c in cases])
    if graph:
        b2.use_graph(graph)
    assert b2.autotune(trial_steps=2, cache_path=cache) == by
    assert b2.launch_config() == cfg
    for i, c in enumerate(cases):
        b.set_fields(i, *c.fields)
    b.step(6)
    ref = _batch(cases)
    ref.step(6)
    for i in range(len(cases)):
        np.testing.assert_array_equal(b.get_f(i), ref.get_f(i))


def test_batch_fp32_per_instance_bases_equal_single_instance_runs_bitwise():
    """FP32 storage with a different departure base per instance (each
    instance's descriptor holds its own base): the batch equals separate
    single-instance runs with the same bases, bitwise, wall densities
    included."""
    olb = _olb()
    cases = _channels(precision=1)
    bases = [0.8 * I.T_CRIT, I.T_CRIT, 1.0]
    b = olb.Batch([c.params for c in cases])
    for i, c in enumerate(cases):
        b.set_base_temperature(i, bases[i])
        b.set_fields(i, *c.fields)
    b.step(7)
    for i, c in enumerate(cases):
        lat = olb.Lattice(c.params)
        lat.set_base_temperature(bases[i])
        lat.set_fields(*c.fields)
        lat.step(7)
        np.testing.assert_array_equal(b.get_f(i), lat.get_f())
        lo, hi = lat.wall_density()
        blo, bhi = b.wall_density(i)
        np.testing.assert_array_equal(blo, lo)
        np.testing.assert_array_equal(bhi, hi)
        lat.close()
    b.close()


def test_batch_fp32_mixed_density_within_1e5():
    cases = _channels(precision=1)
    steps = 10
    b = _batch(cases)
    b.step(steps)
    for i, c in enumerate(cases):
        p64 = dict(c.params)
        p64["precision"] = 0
        c64 = I.Case(c.name, p64, c.n, c.ux, c.uy, c.T, steps)
        err = moment_errors(b.moments(i), _oracle_run(c64, steps))
        print(f"[batch] fp32 {c.name}: {err}", flush=True)
        assert err["n"] < 1e-5, err


def test_batch_specular_boxes_match_oracle_per_instance():
    """Boxes with specular planes at both ends of x, of uneven sizes (one
    narrower than a tile, one with ragged tiles, one three columns wide), in
    one launch per stage."""
    cases = [I.box(70, 20, seed=41, tw=0.75 * I.T_CRIT), I.box(9, 33, seed=42, temperature=I.T_CRIT),
             I.box(3, 15, seed=43, tw=0.9 * I.T_CRIT)]
    steps = 15
    b = _batch(cases)
    b.step(steps)
    b.sync()
    for i, c in enumerate(cases):
        err = moment_errors(b.moments(i), _oracle_run(c, steps))
        print(f"[batch] {c.name}: {err}", flush=True)
        assert max(err.values()) < TOL64, (c.name, err)


def test_full_channels_batch_matches_oracle_on_sampled_instances():
    """The 256-channel FP32 benchmark batch in its launch configuration
    (one launch per stage over all channels, HIP graphs of 10 steps,
    autotuned tile): 20 steps, then the three smallest channels against
    their own oracle runs."""
    cases = I.channels()
    b = _batch(cases, graph=10)
    b.autotune(trial_steps=2)
    for i, c in enumerate(cases):                 # the trial overwrote the fields
        b.set_base_temperature(i, float(np.mean(c.T)))   # as the benchmark runs it
        b.set_fields(i, *c.fields)
    steps = 20
    b.step(steps)
    b.sync()
    small = sorted(range(len(cases)), key=lambda i: cases[i].params["nx"] * cases[i].params["ny"])[:3]
    for i in small:
        c = cases[i]
        err = moment_errors(b.moments(i), _oracle_run(c, steps))
        print(f"[batch] channel {i} ({c.params['nx']}x{c.params['ny']}, T_w {c.params['tw_lo']:.3f}): {err}",
              flush=True)
        assert err["n"] < 1e-5, (i, err)
    b.close()


def test_batch_rejects_mixed_kinds_and_bad_index():
    olb = _olb()
    a = I.shear32().params
    w = I.channel(16, 8).params
    with pytest.raises(olb.OlbError) as e:
        olb.Batch([a, w])
    assert e.value.code == olb.OLB_E_ARG
    # specular x and periodic x cannot share a batch
    with pytest.raises(olb.OlbError) as e:
        olb.Batch([I.box(8, 12).params, I.half_channel(8, 12).params])
    assert e.value.code == olb.OLB_E_ARG
    b = olb.Batch([a])
    with pytest.raises(olb.OlbError) as e:
        b.set_fields(3, *I.shear32().fields)
    assert e.value.code == olb.OLB_E_ARG
