"""The binding refuses vectors the library would read or write out of bounds (no GPU needed).

Each check runs before any pointer reaches the library, so the cases use CPU
tensors: against a CUDA device they must be refused for their device, and
against a CPU device they exercise the dtype, shape and stride rules.
"""
import pytest

torch = pytest.importorskip("torch")

from paper_1712_00403_amd import fd  # noqa: E402

CPU = torch.device("cpu")
N = 10


def test_host_tensors_are_refused_for_a_device_plan():
    r = torch.zeros(2, N, dtype=torch.float64)
    with pytest.raises(ValueError, match="cuda"):
        fd.check_vectors(r, None, N, "float64", torch.device("cuda", 0))
    with pytest.raises(ValueError, match="cuda"):
        fd.check_vectors(r, r.clone(), N, "float64", torch.device("cuda", 0))


def test_dtype_must_be_the_plans():
    r = torch.zeros(2, N, dtype=torch.float64)
    z32 = torch.zeros(2, N, dtype=torch.float32)
    with pytest.raises(TypeError):
        fd.check_vectors(r, z32, N, "float64", CPU)
    with pytest.raises(TypeError):
        fd.check_vectors(z32, None, N, "float64", CPU)


def test_z_must_match_r():
    r = torch.zeros(3, N + 4, dtype=torch.float32)
    fd.check_vectors(r, torch.zeros_like(r), N, "float32", CPU)
    with pytest.raises(ValueError, match="shape"):
        fd.check_vectors(r, torch.zeros(2, N + 4, dtype=torch.float32), N, "float32", CPU)
    with pytest.raises(ValueError, match="shape"):
        fd.check_vectors(r, torch.zeros(3, N, dtype=torch.float32), N, "float32", CPU)
    # same shape, different row stride
    zs = torch.zeros(3, N + 8, dtype=torch.float32)[:, :N + 4]
    with pytest.raises(ValueError, match="strides"):
        fd.check_vectors(r, zs, N, "float32", CPU)


def test_vectors_too_short_or_not_unit_stride():
    with pytest.raises(ValueError, match="entries"):
        fd.check_vectors(torch.zeros(2, N - 1, dtype=torch.float64), None, N, "float64", CPU)
    with pytest.raises(ValueError, match="stride"):
        fd.check_vectors(torch.zeros(N, 2, dtype=torch.float64).t(), None, N, "float64", CPU)
    with pytest.raises(ValueError, match="shape"):
        fd.check_vectors(torch.zeros(2, 2, N, dtype=torch.float64), None, N, "float64", CPU)


def test_block_vectors_must_be_exact_and_contiguous():
    r = torch.zeros(2, N + 1, dtype=torch.float32)
    with pytest.raises(ValueError, match="exactly"):
        fd.check_vectors(r, None, N, "float32", CPU, exact=True)
    fd.check_vectors(torch.zeros(2, N, dtype=torch.float32), None, N, "float32", CPU, exact=True)
    fd.check_vectors(torch.zeros(N, dtype=torch.float32), None, N, "float32", CPU, exact=True)
    fd.check_vectors(torch.zeros(0, N, dtype=torch.float32), None, N, "float32", CPU, exact=True)
