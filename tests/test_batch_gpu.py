"""Batched persistent launches: every instance of a batched run equals the
plain per-instance run bit for bit (same per-block arithmetic), for several
schedules and with HIP-graph replay; sampled instances match the oracle."""
import numpy as np
import pytest
import torch

from oracle.cdg2_oracle import Config, Oracle
from parity_util import TOL, assert_close
from paper_1403_1157_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def small_batch(count=10, seed=9):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = (int(rng.choice([4, 6, 8, 12])), int(rng.choice([4, 5, 8, 10])))
        p = int(rng.integers(1, 4))
        out.append(dict(n=n, order=p, coeffs=inputs.sample_coeffs((99, i)), key=(99, i)))
    return out


def states_for(insts):
    return [torch.from_numpy(inputs.initial_modes(2, it["n"], it["order"], it["key"])).to(DEV)
            for it in insts]


def dts_for(insts, states):
    from paper_1403_1157_amd.cdg2 import Operator
    dts = []
    for it, U in zip(insts, states):
        op = Operator(2, it["n"], it["order"], it["coeffs"])
        dts.append(op.max_dt(U, 0.9))
        op.close()
    return dts


def per_instance(insts, states, dts, nsteps):
    from paper_1403_1157_amd.cdg2 import Operator
    outs = []
    for it, U, dt in zip(insts, states, dts):
        op = Operator(2, it["n"], it["order"], it["coeffs"])
        X = U.clone()
        op.rk_step(X, dt, nsteps)
        op.sync()
        outs.append(X)
    return outs


@pytest.mark.parametrize("schedule", [(32, 0, 0), (16, 64, 1), (64, 8, 0), (32, 3, 1), (32, 0, 2), (16, 5, 2)])
@pytest.mark.parametrize("graph", [False, True])
def test_batched_equals_per_instance(schedule, graph):
    from paper_1403_1157_amd.batch import Batch
    insts = small_batch()
    states = states_for(insts)
    dts = dts_for(insts, states)
    ref = per_instance(insts, states, dts, 3)
    bt = Batch(insts)
    bt.set_schedule(*schedule)
    packed = bt.pack(states)
    bt.rk(packed, dts, 3, graph=graph)
    bt.sync()
    for i in range(len(insts)):
        assert torch.equal(bt.view(packed, i), ref[i]), i
    bt.close()


@pytest.mark.parametrize("graph", [False, True])
def test_caller_offsets_place_instances_anywhere(graph):
    """cdg2_batch_rk with caller offsets (the instances in reverse order inside the
    same packed size) gives the same per-instance results as the library's
    packing; an overlapping or out-of-range placement is rejected."""
    from paper_1403_1157_amd.batch import Batch
    from paper_1403_1157_amd.cdg2 import CDG2_EINVAL, CDG2Error
    insts = small_batch(7, seed=4)
    states = states_for(insts)
    dts = dts_for(insts, states)
    ref = per_instance(insts, states, dts, 2)
    bt = Batch(insts)
    sizes = [s[0] * s[1] * s[2] for s in bt.shapes]
    offs, pos = [0] * len(insts), 0
    for i in reversed(range(len(insts))):
        offs[i] = pos
        pos += sizes[i]
    packed = torch.empty(bt.total, dtype=torch.float64, device=DEV)
    for i, U in enumerate(states):
        packed[offs[i]:offs[i] + sizes[i]] = U.reshape(-1)
    bt.rk(packed, dts, 2, graph=graph, offsets=offs)
    bt.sync()
    for i in range(len(insts)):
        assert torch.equal(packed[offs[i]:offs[i] + sizes[i]].view(bt.shapes[i]), ref[i]), i
    bad = list(offs)
    bad[0] = offs[1]                       # overlaps instance 1
    with pytest.raises(CDG2Error) as ei:
        bt.rk(packed, dts, 1, offsets=bad)
    assert ei.value.code == CDG2_EINVAL
    bad = list(offs)
    bad[2] = bt.total - sizes[2] + 1       # leaves the packed size
    with pytest.raises(CDG2Error) as ei:
        bt.rk(packed, dts, 1, offsets=bad)
    assert ei.value.code == CDG2_EINVAL
    bt.close()


def test_create_with_native_autotune():
    from paper_1403_1157_amd.batch import Batch
    insts = small_batch(6, seed=2)
    states = states_for(insts)
    dts = dts_for(insts, states)
    ref = per_instance(insts, states, dts, 2)
    bt = Batch(insts, autotune=True)
    packed = bt.pack(states)
    bt.rk(packed, dts, 2)
    bt.sync()
    for i in range(len(insts)):
        assert torch.equal(bt.view(packed, i), ref[i]), i
    bt.close()


def test_graph_replays_match_eager():
    """Replay the captured graph several times with eager work and
    synchronisations between replays; every replay equals the eager run."""
    from paper_1403_1157_amd.batch import Batch
    insts = small_batch(6, seed=3)
    states = states_for(insts)
    dts = dts_for(insts, states)
    bt = Batch(insts)
    eager = bt.pack(states)
    graph_state = eager.clone()
    for rep in range(3):
        bt.rk(eager, dts, 2, graph=False)
        bt.sync()
        junk = torch.randn(1000, device=DEV).sum()          # unrelated eager work
        torch.cuda.synchronize()
        bt.rk(graph_state, dts, 2, graph=True)
        bt.sync()
        assert torch.equal(graph_state, eager), rep
    bt.close()


def test_batched_instances_match_oracle():
    from paper_1403_1157_amd.batch import Batch
    insts = small_batch(8, seed=5)
    states = states_for(insts)
    dts = dts_for(insts, states)
    bt = Batch(insts)
    packed = bt.pack(states)
    bt.rk(packed, dts, 4)
    bt.sync()
    for i in (0, 3, 7):
        it = insts[i]
        o = Oracle(Config(dim=2, n=it["n"], order=it["order"], coeffs=it["coeffs"]))
        Uo = o.rk_step(states[i].cpu(), dts[i], 4)
        assert_close(bt.view(packed, i), Uo, TOL["fp64"], f"instance {i}")
    bt.close()


def test_full_batch_sample_and_autotuner(tmp_path):
    """The 256-instance workload (grid sides 32..128, orders 1..3, coefficients
    within +-50%): autotune, run 2 steps, compare 16 sampled instances with their
    plain per-instance runs (bitwise) and one with the oracle."""
    from paper_1403_1157_amd.batch import Batch
    insts = inputs.batch_instances(256)
    states = states_for(insts)
    dts = dts_for(insts, states)
    bt = Batch(insts)
    packed = bt.pack(states)
    best = bt.autotune(cache_path=str(tmp_path / "tune.json"))
    print(f"[batch] autotuned schedule {best['schedule']} {best['ms_per_step']:.3f} ms/step", flush=True)
    assert (tmp_path / "tune.json").exists()
    bt.rk(packed, dts, 2)
    bt.sync()
    sample = list(range(0, 256, 16))
    ref = per_instance([insts[i] for i in sample], [states[i] for i in sample], [dts[i] for i in sample], 2)
    for k, i in enumerate(sample):
        assert torch.equal(bt.view(packed, i), ref[k]), i
    it = insts[17]
    o = Oracle(Config(dim=2, n=it["n"], order=it["order"], coeffs=it["coeffs"]))
    assert_close(bt.view(packed, 17), o.rk_step(states[17].cpu(), dts[17], 2), TOL["fp64"], "oracle sample")
    bt.close()
