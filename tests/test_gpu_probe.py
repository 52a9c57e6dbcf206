"""GPU test of the DFT-16 unit probe: the matrix-core version computes the
16-point DFT of the documented operand layout (which checks the lane
layout of the 16x16x4 FP32 matrix instruction), the vector version returns
its input after forward-then-inverse pairs, and both time."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pmb():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1302_0120_amd import binding
    return binding


def test_probe_matrix_layout_and_vector_round_trip(pmb):
    waves = 8
    rng = np.random.default_rng(16)
    x = (rng.standard_normal(waves * 1024) + 1j * rng.standard_normal(waves * 1024)).astype(np.complex64)
    xd = torch.from_numpy(x).cuda()
    out, ms = pmb.probe_dft16(True, xd, 2)
    # reference: per wave w and block b, Y = F X with X[t][j] = x[1024 w + 256 b + 16 t + j]
    X = x.astype(np.complex128).reshape(waves, 4, 16, 16)
    F = np.exp(-2j * np.pi * np.outer(np.arange(16), np.arange(16)) / 16)
    Y = 2 * np.einsum("kt,wbtj->wbkj", F, X)  # accumulated over the 2 reps
    got = out.cpu().numpy().astype(np.complex128).reshape(waves, 4, 16, 16)
    err = np.linalg.norm(got - Y) / np.linalg.norm(Y)
    print(f"matrix DFT-16 rel L2 {err:.2e}, {ms:.3f} ms", flush=True)
    assert err <= 1e-6 and ms > 0
    back, ms_v = pmb.probe_dft16(False, xd, 2)
    err_v = np.linalg.norm(back.cpu().numpy() - x) / np.linalg.norm(x)
    assert err_v <= 1e-6 and ms_v > 0


@pytest.mark.parametrize("shape", [(1024, 1024), (600, 800), (256, 128)])
def test_exchange_probe_copies_in_place(pmb, shape):
    """The exchange probe runs the plan's passes in copy mode: the buffer
    comes back bitwise unchanged (every element stored where it was loaded,
    by both thread maps), the plan's own solve is unaffected, and the time is
    positive; bad arguments are PM_EINVAL, a batched handle PM_ESTATE."""
    h, w = shape
    print(f"exchange probe {shape}", flush=True)
    rng = np.random.default_rng(h + w)
    x = (rng.standard_normal((h, w)) + 1j * rng.standard_normal((h, w))).astype(np.complex64)
    buf = torch.from_numpy(x).cuda()
    plan = pmb.PhaseMask(h, w)
    ms = plan.probe_exchange(buf, 3)
    assert ms > 0
    assert torch.equal(buf.cpu(), torch.from_numpy(x))
    with pytest.raises(pmb.PhaseMaskError) as ei:
        plan.probe_exchange(buf, 0)
    assert ei.value.status == -1
    bp = pmb.BatchedPhaseMask([(64, 64)])
    import ctypes
    ms_c = ctypes.c_float()
    assert pmb.lib.phasemask_probe_exchange(bp._h, ctypes.c_void_p(buf.data_ptr()), 1, ctypes.byref(ms_c)) == -5
