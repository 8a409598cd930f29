"""The C-ABI library: it loads, exports every function the headers declare, and
its host-only entry points (workspace sizing, configuration checks, parameter
count) behave as documented.  No call here touches a GPU."""
import ctypes
import glob
import os
import re

import pytest

from paper_1306_1821_amd import binding, build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for path in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))):
        text = open(path).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        text = re.sub(r"#[^\n]*", "", text)
        text = re.sub(r"typedef[^;]*;", "", text)
        text = re.sub(r"(struct|enum)\s+\w*\s*\{.*?\}\s*\w*\s*;", "", text, flags=re.S)
        names += re.findall(r"\b([A-Za-z_]\w*)\s*\([^;{}()]*\)\s*;", text)
    return names


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(binding.LIB_PATH):
        build.build()
    return binding.lib()


def test_headers_declare_the_documented_calls():
    names = declared_functions()
    for required in ("hmc_init", "leapfrog_trajectory", "hamiltonian", "shell_power",
                     "gibbs_sweep", "cnn_forward", "cnn_train_step"):
        assert required in names
    assert len(names) == len(set(names))


def test_library_exports_every_declared_function(L):
    names = declared_functions()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(names) == sorted(binding.EXPORTS)


def _cfg(**kw):
    c = binding.HmcConfig()
    c.n, c.box, c.n_sub, c.n_bins = 32, 500.0, 1, 16
    c.alpha_prior, c.seed, c.chain_id, c.n_leapfrog, c.eps = 1.0, 1, 0, 20, 0.05
    c.fixed_bias_mask, c.rj_move, c.rj_log_bound, c.tau_mode = 1, 0, 10.0, 0
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def test_workspace_bytes_valid_and_growing(L):
    sizes = [L.hmc_workspace_bytes(ctypes.byref(_cfg(n=n))) for n in (8, 16, 32, 64, 128, 192, 256)]
    assert all(s > 0 for s in sizes)
    assert all(b > a for a, b in zip(sizes, sizes[1:]))
    # at least the four half-grid complex work grids of a 256^3 chain
    assert sizes[-1] >= 4 * 256 * 256 * 129 * 8


@pytest.mark.parametrize("bad", [dict(n=100), dict(n=4), dict(n_sub=0), dict(n_sub=33),
                                 dict(n_bins=0), dict(n_bins=129), dict(box=0.0),
                                 dict(n_leapfrog=0), dict(eps=0.0), dict(eps=float("inf")),
                                 dict(chain_id=1 << 24)])
def test_workspace_bytes_rejects_invalid_configurations(L, bad):
    assert L.hmc_workspace_bytes(ctypes.byref(_cfg(**bad))) == 0


def test_null_arguments(L):
    assert L.hmc_workspace_bytes(None) == 0
    assert isinstance(L.hmc_last_error(None), bytes)
    assert isinstance(L.cnn_last_error(None), bytes)
    out = ctypes.c_void_p()
    assert L.hmc_init(None, None, None, None, None, None, ctypes.byref(out)) != binding.HMC_OK
    assert L.hamiltonian(None, 0, None) != binding.HMC_OK
    assert L.hmc_set_step(None, 0, 0.1) != binding.HMC_OK
    assert L.hmc_set_plan(None, 0, 0) != binding.HMC_OK
    assert L.hmc_set_mass_diagonal(None, 0, None) != binding.HMC_OK
    assert L.hmc_field_moments(None, 0, None, None, 1) != binding.HMC_OK
    assert L.hmc_get_launch(None, None, None) != binding.HMC_OK
    L.hmc_destroy(None)
    L.cnn_destroy(None)


def test_cnn_parameter_count(L):
    assert L.cnn_param_count() == sum(27 * ci * co + co for ci, co in binding.CNN_LAYERS) == 16034


def test_shell_power_noalloc_rejects_bad_arguments_on_the_host(L):
    """Argument checks come before any device call (no GPU needed)."""
    buf = (ctypes.c_double * 4)()
    assert L.shell_power_noalloc(32, 16, None, buf, None, None) == binding.STATUS_EINVAL
    assert b"null" in L.hmc_last_error(None)
    dummy = ctypes.c_void_p(1)   # never dereferenced: the size checks fail first
    assert L.shell_power_noalloc(48, 16, dummy, buf, None, None) == binding.STATUS_EINVAL
    assert b"N must be" in L.hmc_last_error(None)
    assert L.shell_power_noalloc(32, 0, dummy, buf, None, None) == binding.STATUS_EINVAL
    assert L.shell_power_noalloc(32, 129, dummy, buf, None, None) == binding.STATUS_EINVAL
    assert b"n_bins" in L.hmc_last_error(None)
