"""One coarse step of the subcycled driver captured as a hipGraph of persistent level
solves and replayed (amrfld_opts.graph with persistent): every replay against the same
steps run eagerly (host-polled sweeps, and one persistent launch per solve), bitwise with
equal iteration counts, with the program's own eager work and synchronisations between
the replays; a change of dt, of the fields or of the launch shape forces a new capture.
In mixed precision each captured solve is the whole refinement loop in one persistent
launch, its decisions made on the device."""
import numpy as np
import pytest

from synth.configs import config_collapse, config_equilibrium, config_tiny

pytestmark = pytest.mark.gpu


def _run(p, mode, dts, reset_each=False, **kw):
    from paper_1401_1112_amd.solver import sample_problem_fields, solver_from_problem, to_numpy
    s = solver_from_problem(p, **kw)
    out = []
    for dt in dts:
        if reset_each:
            sample_problem_fields(s, p)
        # Neumann / Robin steps can end with negative energies (Sect. 3.3.5) and the next
        # step's system then may end non-finite: every form must take the same path
        status = s.advance(dt, mode, p.tol, raise_on_error=False)
        st = s.stats()
        out.append(({l: (to_numpy(s.E(l)), None if p.T is None else to_numpy(s.E(l, with_T=True)[1]))
                     for l in p.hierarchy.levels},
                    [status] + [(x["level"], x["iters"]) for x in st], {x["launch_mode"] for x in st}))
    s.close()
    return out


def _same(a, b):
    for (fa, ia, _), (fb, ib, _) in zip(a, b):
        if ia[0] != 0 or ib[0] != 0:
            # a failed step (non-finite after negative energies): the same status; an eager
            # step stops at the failing solve while a replay runs all of them, so nothing
            # after it is compared
            assert ia[0] == ib[0]
            return
        assert ia == ib
        for l in fa:
            assert np.array_equal(fa[l][0], fb[l][0], equal_nan=True)
            if fa[l][1] is not None:
                assert np.array_equal(fa[l][1], fb[l][1], equal_nan=True)


CASES = {
    "tiny_lp": lambda: config_tiny(0, base_level=3, max_level=5, p_refine=0.5, kmode="lp", tol=1e-12),
    "tiny_const": lambda: config_tiny(3, base_level=3, max_level=5, p_refine=0.5, kmode="const", tol=1e-12),
    "coupled": lambda: config_collapse(base_level=3, max_level=7, jeans=2.5, contrast=1e4, field_n=64,
                                       shared_dt_levels=2),
    "equilibrium": lambda: config_equilibrium(max_level=5, tol=1e-12),
}


def _theta_case():
    p = config_tiny(4, base_level=3, max_level=5, p_refine=0.5, kmode="lp", tol=1e-12)
    p.theta = 0.5
    return p


@pytest.mark.parametrize("form_coefs", [False, True])
def test_graph_theta_and_formed_coefficients(form_coefs):
    # the Crank-Nicolson step (Dirichlet interfaces) captured and replayed, with stored
    # or formed face coefficients
    p = _theta_case()
    dts = [p.dt_coarse] * 3
    graph = _run(p, 0, dts, persistent=True, graph=True, form_coefs=form_coefs)
    assert all(m == {2} for _, _, m in graph)
    _same(graph, _run(p, 0, dts))


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_graph_replays_equal_eager(case, mode):
    p = CASES[case]()
    dts = [p.dt_coarse] * 3
    graph = _run(p, mode, dts, persistent=True, graph=True)
    assert all(m == {2} for _, _, m in graph)
    eager = _run(p, mode, dts, persistent=True)
    assert all(m == {1} for _, _, m in eager)
    polled = _run(p, mode, dts)
    _same(graph, eager)
    _same(graph, polled)


def test_graph_recaptures_on_changes():
    # dt changes, then returns; the fields are set anew before every step (set_coeffs)
    p = config_tiny(1, base_level=3, max_level=5, p_refine=0.5, kmode="lp", tol=1e-12)
    dts = [p.dt_coarse, 0.5 * p.dt_coarse, p.dt_coarse, p.dt_coarse]
    _same(_run(p, 0, dts, persistent=True, graph=True), _run(p, 0, dts))
    _same(_run(p, 0, dts, reset_each=True, persistent=True, graph=True), _run(p, 0, dts, reset_each=True))


def test_graph_launch_shape_change_recaptures():
    from paper_1401_1112_amd.solver import solver_from_problem, to_numpy
    p = config_tiny(2, base_level=3, max_level=5, p_refine=0.5, kmode="lp", tol=1e-12)
    res = []
    for graph in (True, False):
        s = solver_from_problem(p, persistent=True, graph=graph)
        s.advance(p.dt_coarse, 0, p.tol)
        s.set_launch(256, True, 1)  # another block count and resident blocks per compute unit
        s.advance(p.dt_coarse, 0, p.tol)
        res.append(({l: to_numpy(s.E(l)) for l in p.hierarchy.levels}, [x["iters"] for x in s.stats()],
                    {x["launch_mode"] for x in s.stats()}))
        s.close()
    assert res[0][2] == {2} and res[1][2] == {1}
    assert res[0][1] == res[1][1]
    assert all(np.array_equal(res[0][0][l], res[1][0][l]) for l in res[0][0])


@pytest.mark.parametrize("case", ["tiny_lp", "coupled"])
@pytest.mark.parametrize("mode", [0, 2])
def test_graph_mixed_replays_equal_eager(case, mode):
    from paper_1401_1112_amd import MIXED
    p = CASES[case]()
    dts = [p.dt_coarse] * 3
    graph = _run(p, mode, dts, precision=MIXED, persistent=True, graph=True)
    assert all(m == {2} for _, _, m in graph)
    eager = _run(p, mode, dts, precision=MIXED, persistent=True)
    assert all(m == {1} for _, _, m in eager)
    polled = _run(p, mode, dts, precision=MIXED)
    _same(graph, eager)
    _same(graph, polled)
