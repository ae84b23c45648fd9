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


@pytest.mark.parametrize("inner_tol", [1e-2, 1e-5])
def test_refinement_split_keeps_the_fp64_threshold(inner_tol):
    # any inner tolerance only moves work between FP32 inner iterations and FP64
    # refinement sweeps: every solve still meets the FP64 stopping rule
    from paper_1401_1112_amd import E_INVALID, MIXED, _lib as L
    from paper_1401_1112_amd.solver import solver_from_problem, to_numpy
    from synth.configs import config_tiny
    p = config_tiny(2, base_level=3, max_level=5, p_refine=0.5, kmode="lp", tol=1e-10)
    ref = solver_from_problem(p)
    ref.advance(p.dt_coarse, 0, p.tol)
    s = solver_from_problem(p, precision=MIXED)
    assert L.amrfld_set_refinement(s.ctx, 0.0, 30) == E_INVALID
    assert L.amrfld_set_refinement(s.ctx, 1e-4, 0) == E_INVALID
    s.set_refinement(inner_tol)
    s.advance(p.dt_coarse, 0, p.tol)
    for st in s.stats():
        thr = max(p.tol * st["rnorm0"], p.abs_floor * st["bnorm"])
        assert st["converged"] == 1 and st["true_rel_res"] * st["rnorm0"] <= thr * (1 + 1e-12), st
    for l in p.hierarchy.levels:
        a, b = to_numpy(s.E(l)), to_numpy(ref.E(l))
        assert np.linalg.norm(a - b) <= 1e-8 * np.linalg.norm(b)
    s.close()
    ref.close()


def test_oversized_batch_rejected_on_every_call():
    # two patches of 1024^3 cells exceed the 32-bit slot space: the layout build fails
    # before any launch, leaves no layout behind, and the same call fails the same way
    # again; a batch that fits then runs on the same context
    import torch
    from paper_1401_1112_amd import E_INVALID, _lib as L
    from paper_1401_1112_amd.solver import BatchSolver
    n = 1024
    rho = torch.ones(n ** 3, dtype=torch.float64, device="cuda")
    E = torch.ones(n ** 3, dtype=torch.float64, device="cuda")
    out = torch.empty(2 * n ** 3, dtype=torch.float64, device="cuda")
    structs = []
    for _ in range(2):
        st = L.amrfld_patch()
        st.n, st.dx, st.dt = n, 1.0 / n, 1e-3
        st.rho, st.E = rho.data_ptr(), E.data_ptr()
        st.kmode, st.K_const, st.kappa_R, st.c_light = L.K_CONST, 1.0, 1.0, 1.0
        structs.append(st)
    patches, alpha = patch_batch(5, 3, n_min=4, n_max=8)
    bs = BatchSolver(robin_alpha=alpha)
    for _ in range(2):
        assert L.amrfld_solve_batch(bs.ctx, structs, 1, 1e-10, 0, out) == E_INVALID
        assert "32-bit" in str(L.amrfld_last_error(bs.ctx))
    del rho, E, out
    torch.cuda.empty_cache()
    h = bs.upload(patches)
    assert bs.run(h, 2, 1e-10) == 0
    assert torch.isfinite(h["out"]).all()
    bs.close()
