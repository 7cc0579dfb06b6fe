"""Argument checks that need no GPU: the Python binding rejects host tensors,
wrong dtypes and particle counts beyond a tensor's view before any call
reaches the library, and the stage integrator's Newton-step count."""
import numpy as np
import pytest
import torch



@pytest.fixture(scope="module")
def hbl():
    from paper_2402_17248_amd import hbl as h
    return h


def test_host_tensor_rejected(hbl):
    z = torch.zeros((6, 8), dtype=torch.float64)
    with pytest.raises(ValueError, match="device tensor"):
        hbl.fill_gaussian(z, 1, (0.0,) * 6, (1.0,) * 6)
    with pytest.raises(ValueError, match="device tensor"):
        hbl.moments(z)
    with pytest.raises(ValueError, match="device tensor"):
        hbl.compare(z, z)


def test_wrong_dtype_and_layout_rejected(hbl):
    with pytest.raises(TypeError):
        hbl.moments(torch.zeros((6, 8), dtype=torch.int64))
    with pytest.raises(TypeError):
        hbl.moments(torch.zeros((8, 6), dtype=torch.float64).t())
    with pytest.raises(TypeError):
        hbl.moments(np.zeros((6, 8)))


@pytest.mark.parametrize("n", [-1, 9, 100])
def test_count_beyond_view_rejected(hbl, n):
    base = torch.zeros((6, 16), dtype=torch.float64)
    view = base[:, 4:12]                    # 8 particles inside a wider allocation
    with pytest.raises(ValueError, match="outside"):
        hbl.fill_gaussian(view, 1, (0.0,) * 6, (1.0,) * 6, n=n)


def test_moments_output_must_be_device_float64(hbl):
    with pytest.raises(ValueError, match="device tensor"):
        hbl._out27_arg(torch.zeros(27, dtype=torch.float64))


def test_index_bounds(hbl):
    assert list(hbl._index_args([0, 5, 9], 10, "t")) == [0, 5, 9]
    for bad in ([0, 10], [-1]):
        with pytest.raises(ValueError):
            hbl._index_args(bad, 10, "t")


@pytest.mark.parametrize("nsub,steps", [(1000, 4), (1297, 4), (1453, 4), (1609, 3), (2000, 3), (32000, 3), (400000, 2), (40, 0)])
def test_newton_steps_stage1(hbl, nsub, steps):
    """Stage 1 of the chain (1 -> 11 GeV over 0.3 m): the reciprocal of gamma
    changes per substep by d = ramp/(0.9 gamma_in); k Newton steps leave
    d^(2^k), the fewest k <= 4 with d^(2^k) < 1e-17 is used, else a divide."""
    ref = hbl.Ref.from_energy(1000.0)
    g_in = ref.gamma
    g_out = g_in + 10000.0 / hbl.MEC2_MEV
    d = (g_out - g_in) / nsub / (0.9 * g_in)
    want = next((k for k in range(1, 5) if d ** (2 ** k) < 1e-17), 0)
    assert want == steps
    st = hbl.Element(hbl.STAGE, nsub, 0.3, 0.0, 0.0, 0.0, 1e23, 10000.0, 0.0, 0, 0)
    assert hbl.stage_newton_steps(st, ref) == steps
