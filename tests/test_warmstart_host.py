"""Host-side pieces of the warm-start pipeline (no GPU): the weight file
format and the relative error used for the gate."""
import numpy as np

from paper_2311_05091_amd import warmstart as W


def test_weight_file_round_trip(tmp_path):
    rng = np.random.default_rng(2)
    flat = {"gate": np.array(0.125)}
    ref = {}
    for name, shape in (("e0a", (32, 3, 3, 32)), ("head", (32,))):
        w = rng.normal(size=shape).astype(np.float32)
        b = rng.normal(size=shape[:1] if name != "head" else (1,)).astype(np.float32)
        flat[name + ".w"], flat[name + ".b"] = w, b
        ref[name] = (w, b)
    path = str(tmp_path / "w.npz")
    np.savez_compressed(path, **flat)
    params, gate = W.load_params(path)
    assert gate == 0.125 and set(params) == set(ref)
    for k, (w, b) in ref.items():
        assert np.array_equal(params[k][0], w) and np.array_equal(params[k][1], b)
        assert params[k][0].dtype == np.float64


def test_rel_l2():
    a = np.array([3.0, 4.0])
    assert W.rel_l2(a, a) == 0.0
    assert abs(W.rel_l2(np.zeros(2), a) - 1.0) < 1e-15
    assert abs(W.rel_l2(a * 1.1, a) - 0.1) < 1e-12
