"""Sampler configuration (host logic, no GPU): YAML and dict forms, the
batch-size / flows-per-batch rule, and the checks on optional steps."""

import numpy as np
import pytest

from paper_2512_09664_amd.sampler import FlowProvider, SamplerConfig


def test_yaml_and_dict_forms(tmp_path):
    p = tmp_path / "cfg.yaml"
    p.write_text(
        "image_shape: [256, 320]\n"
        "batch_size: 8\n"
        "flows_per_batch: 4\n"
        "batches_per_flow: 3\n"
        "seeding_density: [0.01, 0.05]\n"
        "diameter: {dist: normal, mean: 2.5, std: 0.5, clip: [1.0, 5.0]}\n"
        "blur: {radius: 1, sigma: 0.7}\n"
        "noise_sigma: 0.01\n"
        "bits: 12\n"
        "flow: {kind: fourier, grid_div: 4, max_disp: 6.0}\n")
    c = SamplerConfig.from_any(str(p))
    assert c.image_shape == [256, 320] and c.batch_size == 8 and c.flows_per_batch == 4
    assert c.d_dist == "normal" and c.d_params == (2.5, 0.5, 1.0, 5.0) and c.d_max == 5.0
    assert c.isotropic
    d = SamplerConfig.from_any({"batch_size": 4, "rho": [-0.5, 0.5], "hide_p": 0.1})
    assert not d.isotropic and d.d_params == (0.8, 1.2)


@pytest.mark.parametrize("bad", [
    {"batch_size": 6, "flows_per_batch": 4},
    {"batches_per_flow": 0},
    {"particle_reuse": {"dt": 1.0, "batches": 3}, "batches_per_flow": 1},
    {"histogram": [1, 2, 3], "bits": 0},
    {"no_such_key": 1},
])
def test_invalid_configurations(bad):
    with pytest.raises(ValueError):
        SamplerConfig.from_any(bad)


def test_flow_provider_shapes_and_epochs(tmp_path):
    fp = FlowProvider({"kind": "lamb_oseen", "grid_div": 4, "max_disp": 8.0}, 128, 96, 3, 7)
    a, b = fp.grids(0), fp.grids(1)
    assert a.shape == (3, 32, 24, 2) and a.dtype == np.float32
    assert not np.array_equal(a, b) and np.array_equal(a, fp.grids(0))
    # the largest node displacement is the configured one
    assert abs(np.hypot(a[0, ..., 0], a[0, ..., 1]).max() - 8.0) < 1e-4
    stack = np.random.default_rng(0).normal(size=(5, 8, 10, 2)).astype(np.float32)
    np.save(tmp_path / "f.npy", stack)
    fq = FlowProvider({"kind": "npy", "path": str(tmp_path / "f.npy")}, 32, 40, 2, 0)
    assert np.array_equal(fq.grids(2), stack[[4, 0]])
    fc = FlowProvider({"fn": lambda e, F, H, W: np.full((F, 4, 5, 2), e, np.float32)}, 16, 20, 2, 0)
    assert np.all(fc.grids(3) == 3.0)
