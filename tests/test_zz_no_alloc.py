"""The allocation-free shell sums (shell_power_noalloc) against shell_power.

Two calls in a row on one GPU, the second on a smaller grid, each compared with
the context entry point on the same field (bit for bit: both run the same tile
and column-sum code) and with the oracle's shell sums."""
import numpy as np
import pytest

from gpu_common import plain_mock
from oracle import grid

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1306_1821_amd import binding  # noqa: E402
from paper_1306_1821_amd.binding import Sampler  # noqa: E402


def field(n, seed):
    rng = np.random.default_rng(seed)
    h = n // 2 + 1
    return (rng.standard_normal((n, n, h)) + 1j * rng.standard_normal((n, n, h))).astype(np.complex64)


@pytest.mark.parametrize("sizes", [[(64, 500.0, 20), (32, 500.0, 16), (256, 1500.0, 128)]])
def test_noalloc_shell_power_matches_context_entry_point(sizes):
    for call, (n, box, nb) in enumerate(sizes):
        mk = plain_mock(n, box, nb)
        s = Sampler([dict(n=n, box=box, nb=nb, R=mk["R"], counts=mk["counts"], bias=mk["bias"],
                          nbar=mk["nbar"], pk=mk["pk_init"])])
        dk = field(n, 100 + call)
        t = s.tensors(0)["delta_k"]
        t.copy_(torch.as_tensor(dk))
        ref_sigma, ref_nm = s.shell_power(0)
        sigma = torch.full((nb,), -1.0, dtype=torch.float64, device="cuda")
        nm = torch.full((nb,), -1, dtype=torch.int64, device="cuda")
        binding.shell_power_noalloc(t, nb, sigma, nm)
        torch.cuda.synchronize()
        got_s, got_n = sigma.cpu().numpy(), nm.cpu().numpy()
        print(f"call {call}: N={n} nb={nb} sigma max rel diff "
              f"{np.max(np.abs(got_s / ref_sigma - 1)):.2e}", flush=True)
        assert np.array_equal(got_s, ref_sigma)
        assert np.array_equal(got_n, ref_nm)
        assert np.array_equal(got_n, grid.mode_counts(n, nb))
        np.testing.assert_allclose(got_s, grid.shell_sums(dk.astype(np.complex128), nb), rtol=1e-12)
        s.close()
