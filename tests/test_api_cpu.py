"""Host-side checks of the torch binding that need no GPU."""
import pytest

torch = pytest.importorskip("torch")

from paper_1712_04732_amd.api import _check_out  # noqa: E402

DEV = torch.device("cpu")


def test_check_out_accepts_matching_outputs():
    N = 7
    _check_out((torch.empty(N), torch.empty(N, 3), torch.empty((), dtype=torch.float64)), N, torch.float32,
               DEV, ())
    _check_out((None, torch.empty(N, 3, dtype=torch.float64), None), N, torch.float64, DEV, ())
    _check_out((None, None, torch.empty(4, dtype=torch.float64)), N, torch.float32, DEV, (4,))


@pytest.mark.parametrize("bad", ["short_phi", "dtype_phi", "short_force", "noncontig", "energy_dtype",
                                 "energy_shape", "not_tensor"])
def test_check_out_rejects_mismatched_outputs(bad):
    """The kernels write N rows of the plan's dtype without bounds checks: a
    short, wrongly typed or strided output must be refused on the host."""
    N = 9
    phi, f, e = torch.empty(N), torch.empty(N, 3), torch.empty((), dtype=torch.float64)
    if bad == "short_phi":
        phi = torch.empty(N - 1)
    elif bad == "dtype_phi":
        phi = torch.empty(N, dtype=torch.float64)
    elif bad == "short_force":
        f = torch.empty(N - 2, 3)
    elif bad == "noncontig":
        f = torch.empty(3, N).t()
    elif bad == "energy_dtype":
        e = torch.empty((), dtype=torch.float32)
    elif bad == "energy_shape":
        e = torch.empty(2, dtype=torch.float64)
    elif bad == "not_tensor":
        phi = [0.0] * N
    with pytest.raises(ValueError):
        _check_out((phi, f, e), N, torch.float32, DEV, ())
