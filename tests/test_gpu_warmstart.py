"""What the learned warm start gains: a network trained briefly on the GPU
(its own kernels) on solver-generated pairs at 32 x 32 (fields up to 128 x 128
block-averaged to 32 x 32, labelled with the block average of their converged
pressure) must start held-out 128 x 128 problems, through the 4x coarsened
grid, closer to the converged pressure than the linear profile does, so that
the unchanged pressure iteration needs fewer sweeps to reach the same
stopping tolerance."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_trained_network_reduces_pressure_iterations():
    from paper_1808_07554_amd import lbtp, warmstart as ws
    size, fine = 32, 128
    lnK, S, P, _ = ws.training_set(768, size, 1_000_000, factors=(1, 2, 4), log=False)
    net = lbtp.WarmStartNet(32, 4, 3.2)
    net.set_params(ws.init_params(32, 4, seed=0))
    losses = ws.train(net, lnK, S, P, 400, 32, 1e-3, log_every=0, weight=ws.relative_weights(P))
    assert np.mean(losses[-20:]) < 0.2 * np.mean(losses[:20])
    eK, eS, ephi = ws.fields(16, fine, 7_000_000)
    r = ws.evaluate(net, eK, eS, ephi, fine // size, starts=("linear", "network"))
    cold, warm = r["starts"]["linear"], r["starts"]["network"]
    print(f"{fine}^2: linear {cold['iterations_mean']:.0f} network {warm['iterations_mean']:.0f} iterations "
          f"(ratio {warm['iteration_ratio']:.2f}, fewer on {warm['fewer_iterations_fraction']:.0%} of fields)")
    assert warm["iteration_ratio"] > 1.15
    assert warm["fewer_iterations_fraction"] >= 0.75
