"""mpdata_mass_noalloc: the mass of mpdata_mass without a context, its
partials in the library's fixed device scratch instead of a workspace.

Checked through the C ABI against mpdata_mass on the same arrays (same
kernels, same block count: bitwise equal) on two calls in a row, the second
with a smaller grid (the scratch keeps the first call's contents), in FP64
and FP32, and against the oracle's compensated sum (2e-16 relative)."""
import numpy as np
import pytest

from paper_1507_01265_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1507_01265_amd import _lib
    _lib.load()


def _noalloc(dtype_code, psi, h):
    from paper_1507_01265_amd import _lib
    out = torch.full((1,), float("nan"), dtype=torch.float64, device=psi.device)
    stream = torch.cuda.current_stream(psi.device)
    _lib.mpdata_mass_noalloc(dtype_code, psi.data_ptr(), h.data_ptr(), psi.numel(),
                             out.data_ptr(), stream.cuda_stream)
    torch.cuda.synchronize()
    return float(out.item())


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["fp64", "fp32"])
def test_noalloc_mass_equals_mass_on_two_calls(orc, dtype):
    from paper_1507_01265_amd import _lib
    from paper_1507_01265_amd.solver import Solver
    code = _lib.MPDATA_FP64 if dtype == torch.float64 else _lib.MPDATA_FP32
    np_dtype = np.float64 if dtype == torch.float64 else np.float32
    for shape, seed in (((13, 45, 70), 501), ((9, 17, 20), 502)):  # second call smaller
        f = inputs.random_smooth(seed, shape).astype(np_dtype)
        s = Solver.from_numpy(f, dtype=dtype)
        s.step(3)
        want = s.mass()
        got = _noalloc(code, s.psi, s.h)
        print(f"noalloc {dtype} {shape}: {got!r} vs mpdata_mass {want!r}", flush=True)
        assert got == want
        ref = orc.mass(s.psi.cpu().numpy().astype(np.float64), f.h.astype(np.float64))
        assert abs(got - ref) <= 2e-16 * abs(ref)
        s.close()


def test_noalloc_mass_empty_and_errors():
    from paper_1507_01265_amd import _lib
    psi = torch.ones(8, dtype=torch.float64, device="cuda")
    h = torch.ones(8, dtype=torch.float64, device="cuda")
    out = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    _lib.mpdata_mass_noalloc(_lib.MPDATA_FP64, psi.data_ptr(), h.data_ptr(), 0, out.data_ptr(), st)
    torch.cuda.synchronize()
    assert out.item() == 0.0
    lib = _lib.load()
    bad = [(5, psi.data_ptr(), h.data_ptr(), 8, out.data_ptr()),
           (0, None, h.data_ptr(), 8, out.data_ptr()),
           (0, psi.data_ptr(), None, 8, out.data_ptr()),
           (0, psi.data_ptr(), h.data_ptr(), 8, None),
           (0, psi.data_ptr(), h.data_ptr(), -1, out.data_ptr()),
           (0, psi.data_ptr(), h.data_ptr(), 2 ** 31, out.data_ptr())]
    for args in bad:
        assert lib.mpdata_mass_noalloc(*args, st) == _lib.MPDATA_EINVAL, args
