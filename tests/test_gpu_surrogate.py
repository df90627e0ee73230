"""The learned-surrogate pipeline on the 160 px sensor at reduced size:
data from the plain kernels, training of the correction network on the GPU,
comparison with the linear interaction-matrix method (the method without the
network), fallback."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_surrogate_beats_linear_interaction_matrix_and_falls_back():
    from paper_2602_06688_amd.surrogate import SurrogatePipeline
    from workloads import workload
    from workloads.modes import coefficient_sigmas, kl_modes
    w = workload("cfg5")
    s = w.sensors[0]
    ex = w.extra
    modes, ev = kl_modes(s.n_pupil, s.obstruction, s.diameter_m, w.L0_m, ex["n_modes"])
    sig = coefficient_sigmas(ev, ex["residual_rms_nm"], s.lambdas_nm[0])
    pipe = SurrogatePipeline(s, modes, sig)
    print("[gpu] surrogate: generating 40k train / 4k test samples", flush=True)
    z, S = pipe.generate(40960, seed=5)
    zt, St = pipe.generate(4096, seed=6)
    print("[gpu] surrogate: interaction matrix and training", flush=True)
    pipe.interaction_matrix()
    e_lin = pipe.rel_error(pipe.linear_predict(zt), St)
    rep = pipe.train(z, S, epochs=12, batch=1024, lr=1e-3)
    e_nn = pipe.rel_error(pipe.predict(zt), St)
    print(f"      linear IM {e_lin:.3e}, surrogate {e_nn:.3e}, losses {rep.losses[0]:.3e}->{rep.losses[-1]:.3e}",
          flush=True)
    assert rep.losses[-1] < rep.losses[0]
    # the network must remove a real part of what the linear model misses:
    # observed 6.16e-2 against 8.46e-2 for the linear model at this size
    # (0.73 of it); the bound holds that figure with a small margin
    assert e_nn < 0.85 * e_lin
    assert e_nn < 0.065
    # fallback: rows far outside the training distribution go to the plain sensor
    zz = zt[:64].clone()
    zz[::4] *= 3.0
    out, mask = pipe.predict_with_fallback(zz)
    ref = pipe.slopes_of(zz)
    m = mask.cpu().numpy()
    assert m[::4].all() and not m[1::4].any()
    assert torch.equal(out[mask], ref[mask])
