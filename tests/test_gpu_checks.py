"""Argument checks that need a device: caller arrays that kernels read or write must be
device memory, and host arrays are rejected with AMRFLD_E_INVALID before any launch
(the context stays usable)."""
import numpy as np
import pytest

from synth.configs import config_uniform, patch_batch

pytestmark = pytest.mark.gpu


def test_host_arrays_rejected_for_levels():
    from paper_1401_1112_amd import E_INVALID, _lib as L
    from paper_1401_1112_amd.solver import solver_from_problem, to_numpy
    p = config_uniform(3, kmode="const")
    s = solver_from_problem(p)
    n = s.info(3)[0]
    host = np.ones(n)
    before = to_numpy(s.E(3)).copy()
    assert L.amrfld_set_coeffs(s.ctx, 3, host, host) == E_INVALID
    assert "device" in str(L.amrfld_last_error(s.ctx))
    assert L.amrfld_get_E(s.ctx, 3, host) == E_INVALID
    assert np.array_equal(to_numpy(s.E(3)), before)
    s.advance(p.dt_coarse, 0, 1e-10)  # still usable
    assert s.stats()[0]["converged"] == 1
    s.close()


def test_host_arrays_rejected_for_patches():
    import torch
    from paper_1401_1112_amd import E_INVALID, _lib as L
    from paper_1401_1112_amd.solver import BatchSolver
    patches, alpha = patch_batch(11, 2, n_min=4, n_max=8)
    bs = BatchSolver(robin_alpha=alpha)
    h = bs.upload(patches)
    host = np.ones(patches[0].n ** 3)
    bad = h["structs"][0]
    keep_rho = bad.rho
    bad.rho = host.ctypes.data
    assert L.amrfld_solve_batch(bs.ctx, h["structs"], 1, 1e-10, 0, h["out"]) == E_INVALID
    bad.rho = keep_rho
    out_host = np.zeros(sum(p.n ** 3 for p in patches))
    assert L.amrfld_solve_batch(bs.ctx, h["structs"], 1, 1e-10, 0, out_host) == E_INVALID
    assert bs.run(h, 1, 1e-10) == 0  # still usable
    assert torch.isfinite(h["out"]).all()
    bs.close()
