"""Call-order and failure paths of the C ABI on the GPU: checkpoints belong to the
media and absorbing layer they were taken with, the non-finite sentinel of loss_step,
and step counts served by the power-of-two step graphs.  No case faults the device: the
NaN is an ordinary float value planted with loss_set_field."""
import numpy as np
import pytest

from gpu_util import announce, require_gpu

pytestmark = pytest.mark.gpu

ESTATE, EUNSUPPORTED, EUNSTABLE = -4, -5, -6


def _acoustic(nsteps, flags=0):
    from paper_2301_05127_amd import inputs, loss
    w = inputs.config("cfg1", nsteps=nsteps)
    sim = loss.Simulation(w["grid"], 0, w["dt"], nshots=1, trace_len=nsteps, flags=flags)
    sim.setup_workload(w)
    return sim, w


def _status_of(fn):
    from paper_2301_05127_amd import loss
    with pytest.raises(loss.LossError) as ei:
        fn()
    return ei.value.status


def test_adjoint_refuses_checkpoints_of_another_layer():
    require_gpu()
    announce("adjoint after set_pml / set_media between forward_ckpt and adjoint")
    sim, w = _acoustic(30)
    res = np.zeros(sim.get_traces(0).size)
    # no layer at the checkpoints, a layer at the adjoint
    sim.forward_ckpt(30, 10)
    sim.set_pml(8, 1e-6, 1.0, 15.0)
    assert _status_of(lambda: sim.adjoint(res)) == ESTATE
    # a layer at the checkpoints, none at the adjoint
    sim.forward_ckpt(30, 10)
    sim.set_pml(0)
    assert _status_of(lambda: sim.adjoint(res)) == ESTATE
    # new media after the checkpoints
    sim.forward_ckpt(30, 10)
    sim.set_media(w["vp"] * 1.01, w["rho"])
    assert _status_of(lambda: sim.adjoint(res)) == ESTATE
    # matching checkpoints run
    sim.forward_ckpt(30, 10)
    g = sim.adjoint(res)
    assert np.isfinite(g).all()
    sim.close()


def test_elastic_adjoint_refuses_layer_added_after_checkpoints():
    require_gpu()
    from paper_2301_05127_amd import inputs, loss
    announce("elastic adjoint with a layer added after forward_ckpt")
    g = inputs.grid(3, (24, 24, 24), (10.0, 10.0, 10.0), (12, 12, 12), 6)
    shape = inputs.field_shape(g)
    sim = loss.Simulation(g, 1, 1e-3, nshots=1, trace_len=8)
    sim.set_media(np.full(shape, 3000.0), np.full(shape, 2200.0), np.full(shape, 1730.0))
    sim.add_source(0, loss.SRC_EXPLOSIVE, (120.0, 120.0, 120.0), inputs.ricker(25.0, 0.048, 1e-3, 9, 0.5), 20.0)
    sim.add_receivers(0, np.array([[12, 12, 4]]), loss.F_EV3)
    sim.forward_ckpt(8, 4)
    sim.set_pml(4, 1e-6, 1.0, 25.0)
    assert _status_of(lambda: sim.adjoint(np.zeros(8))) in (ESTATE, EUNSUPPORTED)
    sim.close()


def test_nonfinite_sentinel():
    require_gpu()
    from paper_2301_05127_amd import loss
    announce("non-finite sentinel: NaN planted with set_field")
    sim, w = _acoustic(64)
    sim.step(3)
    sim.sync()
    f = sim.get_field(loss.F_V3)
    f[40, 70] = np.nan
    sim.set_field(loss.F_V3, f)
    sim.step(2)                      # queued; the check runs after these steps
    assert _status_of(sim.sync) == EUNSTABLE
    assert _status_of(lambda: sim.step(1)) == EUNSTABLE
    sim.reset()
    sim.step(5)
    sim.sync()
    assert np.isfinite(sim.get_field(loss.F_SIGMA)).all()
    sim.close()


@pytest.mark.parametrize("counts", [(1,), (3, 5), (20,), (7, 33, 1)])
def test_graph_step_counts_match_eager(counts):
    """Any sequence of step counts replayed from the power-of-two graphs gives the bits
    of eager launches."""
    require_gpu()
    from paper_2301_05127_amd import loss
    announce("graph step counts %s" % (counts,))
    total = sum(counts)
    a, _ = _acoustic(total)
    b, _ = _acoustic(total, flags=loss.FLAG_NO_GRAPH)
    for c in counts:
        a.step(c)
        b.step(c)
    for f in range(3):
        assert np.array_equal(a.get_field(f), b.get_field(f)), f
    assert np.array_equal(a.get_traces(0), b.get_traces(0))
    a.close()
    b.close()
