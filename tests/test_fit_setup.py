"""Host-side fitting set-up of the package (paper_2605_04017_amd.fit):
parameter layout, initial distribution and the normalisation frame, checked
against the oracle's definitions and closed forms (no GPU)."""
import numpy as np

import synth
from oracle import mlp
from paper_2605_04017_amd import fit as F


def test_param_layout_matches_the_library_order():
    for width, depth, heads in ((128, 5, 1), (64, 4, 3), (32, 2, 56)):
        v = F.init_params(width, depth, heads, 1)
        assert v.dtype == np.float32
        desc = mlp.MapDesc(width, depth, heads, mlp.ACT_TANH)
        assert v.size == mlp.n_params(desc)
        assert F.layer_shapes(width, depth, heads) == mlp.layer_shapes(desc)
        # biases are zero, weights within the Glorot limit and spread over it
        k = 0
        for n_out, n_in in F.layer_shapes(width, depth, heads):
            w, b = v[k:k + n_out * n_in], v[k + n_out * n_in:k + n_out * n_in + n_out]
            lim = np.sqrt(6.0 / (n_out + n_in))
            assert np.all(b == 0) and np.abs(w).max() <= lim
            if w.size > 1000:
                assert abs(w.std() - lim / np.sqrt(3)) < 0.05 * lim
            k += n_out * n_in + n_out
        assert np.array_equal(v, F.init_params(width, depth, heads, 1))


def test_map_norms_are_standardising():
    rays = synth.config_rays(2, 10000)
    ok = np.arange(10000) % 3 == 0
    reg = np.stack([np.linspace(-1, 1, ok.sum())] * 4 + [np.full(ok.sum(), 0.5)], 1)
    in_shift, in_scale, out_shift, out_scale = F.map_norms(rays, [(ok, reg)])
    x = np.stack([rays[k] for k in ("x", "y", "dx", "dy", "dz", "lambda_nm")], 1).astype(np.float64)
    z = (x - in_shift) * in_scale
    assert np.allclose(z.mean(0), 0, atol=1e-9) and np.allclose(z.std(0), 1, atol=1e-9)
    assert np.allclose(out_shift[0, :4], 0, atol=1e-12) and out_scale[0, 4] == 1.0


def test_paper_lr_schedule():
    """Sec. 5.1: 1e-4 decaying by 0.95 every 10,000 batches."""
    from paper_2605_04017_amd import fit as F
    assert F.paper_lr(0) == 1e-4
    assert abs(F.paper_lr(10000) - 0.95e-4) < 1e-18
    assert abs(F.paper_lr(20000) - 0.95 ** 2 * 1e-4) < 1e-18
    assert abs(F.paper_lr(5000) - 0.95 ** 0.5 * 1e-4) < 1e-18
    assert F.paper_lr(395480) < F.paper_lr(395479)
