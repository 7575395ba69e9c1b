"""The on-GPU generator reproduces the host generator bit for bit."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("spec", [
    synth.WORKLOADS[0],
    synth.tiny(seed=41, n_stars=500, obs=(50, 150), n_dfa=700, n_instr_cols=300),
    synth.tiny(seed=42, n_stars=300, obs=(90, 110), n_dfa=900, n_instr_cols=2000,
               value_dtype="f32", astro_scale=(-2.0, 2.0)),
    synth.tiny(seed=43, n_stars=300, obs=(20, 60), n_dfa=150, n_instr_cols=23,
               astro_corr=0.999, n_glob=3, n_instr=4),
], ids=["c0", "uneven", "f32_scaled", "correlated_sections"])
def test_device_generator_is_bit_identical(torch_cuda, spec):
    torch = torch_cuda
    print(f"generator twin: seed={spec.seed} dtype={spec.value_dtype}", flush=True)
    host = synth.make_system(spec)
    dev, first = synth.device_system(spec, "cuda:0")
    torch.cuda.synchronize()
    assert np.array_equal(first, host.first_row)
    assert np.array_equal(dev["star_of_row"].cpu().numpy(), host.star_of_row)
    assert np.array_equal(dev["att_start"].cpu().numpy(), host.att_start)
    assert np.array_equal(dev["instr_idx"].cpu().numpy(), host.instr_idx)
    assert np.array_equal(dev["values"].cpu().numpy().view(np.uint8),
                          host.values.view(np.uint8))
    xt = synth.device_x_true(spec).cpu().numpy()
    assert np.array_equal(xt.view(np.uint64), synth.x_true(spec).view(np.uint64))
    nz = synth.device_noise(spec, host.m, rhs=2).cpu().numpy()
    assert np.array_equal(nz.view(np.uint64), synth.noise(spec, host.m, rhs=2).view(np.uint64))


def test_device_generator_full_size_prefix(torch_cuda):
    # the 1e8-row workload: sampled row ranges against the host generator
    torch = torch_cuda
    spec = synth.WORKLOADS[1]
    print("generator twin: 1e8-row workload, sampled rows", flush=True)
    dev, first = synth.device_system(spec, "cuda:0")
    m = int(first[-1])
    for r0 in (0, 12_345_678, m - 100_000):
        r1 = r0 + 100_000
        v, s, a, i = synth.rows(spec, first, r0, r1)
        assert np.array_equal(dev["values"][:, r0:r1].cpu().numpy(), v)
        assert np.array_equal(dev["star_of_row"][r0:r1].cpu().numpy(), s)
        assert np.array_equal(dev["att_start"][r0:r1].cpu().numpy(), a)
        assert np.array_equal(dev["instr_idx"][:, r0:r1].cpu().numpy(), i)
    del dev
    torch.cuda.empty_cache()
