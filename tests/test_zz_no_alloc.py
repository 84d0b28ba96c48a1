"""The no-allocation solve entry point (bidomain_pcg_solve_noalloc) against bidomain_pcg_solve:
the same kernels in the same order, so the solution and the solve information must be identical,
and both must meet the oracle bar (true relative residual <= 1e-8, relative error <= 1e-6 against
the oracle's rtol-1e-12 solution).  Two calls in a row, the second on a smaller hierarchy, so that
the shared scratch array holds the first call's (larger) contents when the second starts."""
import numpy as np
import pytest

import bidomain_cases as bc
from oracle import amg, fem, krylov

pytestmark = pytest.mark.gpu

lib = pytest.importorskip("paper_2311_13914_amd")


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _problem(dims, seed):
    c = bc.make_case(*dims, seed=seed)
    ops = fem.assemble_operators(c)
    f = -(ops["Ai"] @ bc.nodal_v0(c))
    ref = krylov.amg_pcg(ops["Aell"], f, amg.setup(ops["Aell"], amg.AMGOptions(nullspace=True)), rtol=1e-12,
                         m=ops["m"])
    return c, ops, f, ref.x


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_solve_equals_pcg_solve(torch, prec):
    p = lib.BD_F32 if prec == "f32" else lib.BD_F64
    problems = [_problem((16, 16, 8), 1), _problem((7, 5, 3), 2)]   # the second is smaller
    handles = [lib.bidomain_amg_setup(ops["Aell"], lib.bidomain_default_opts(nullspace=1, vcycle_precision=p), ops["m"])
               for _, ops, _, _ in problems]
    try:
        for (c, ops, f, xref), h in zip(problems, handles):
            print(f"[gpu] noalloc solve n={c.n} {prec}", flush=True)
            b = torch.tensor(f, dtype=torch.float64, device="cuda")
            x1 = torch.zeros(c.n, dtype=torch.float64, device="cuda")
            x2 = torch.full((c.n,), 7.0, dtype=torch.float64, device="cuda")
            rc2, info2 = lib.bidomain_pcg_solve_noalloc(h, b, x2, False, 1e-8, 200)
            rc1, info1 = lib.bidomain_pcg_solve(h, b, x1, False, 1e-8, 200)
            assert rc1 == rc2 == lib.BD_OK
            assert info1["iterations"] == info2["iterations"] > 0
            assert info1["rel_residual_true"] == info2["rel_residual_true"]
            assert info1["rel_residual_rec"] == info2["rel_residual_rec"]
            xs1, xs2 = x1.cpu().numpy(), x2.cpu().numpy()
            assert np.array_equal(xs1, xs2)
            A = ops["Aell"]
            fh = f - f.mean()
            assert np.linalg.norm(fh - A @ xs2) <= 1e-8 * np.linalg.norm(fh)
            assert np.linalg.norm(xs2 - xref) <= 1e-6 * np.linalg.norm(xref)
        # a warm start through the no-allocation call converges at once, as through the other
        c, ops, f, _ = problems[1]
        b = torch.tensor(f, dtype=torch.float64, device="cuda")
        x = torch.zeros(c.n, dtype=torch.float64, device="cuda")
        lib.bidomain_pcg_solve_noalloc(handles[1], b, x, False, 1e-10, 200)
        rc, info = lib.bidomain_pcg_solve_noalloc(handles[1], b, x, True, 1e-8, 200)
        assert rc == lib.BD_OK and info["iterations"] == 0
    finally:
        for h in handles:
            lib.bidomain_amg_destroy(h)


def test_noalloc_rejects_a_solve_larger_than_its_scratch(torch, monkeypatch):
    c, ops, f, _ = _problem((7, 5, 3), 2)
    h = lib.bidomain_amg_setup(ops["Aell"], lib.bidomain_default_opts(nullspace=1), ops["m"])
    try:
        b = torch.tensor(f, dtype=torch.float64, device="cuda")
        x = torch.zeros(c.n, dtype=torch.float64, device="cuda")
        monkeypatch.setenv("BIDOMAIN_NOALLOC_SCRATCH_BYTES", "256")
        with pytest.raises(lib.BidomainError) as e:
            lib.bidomain_pcg_solve_noalloc(h, b, x, False, 1e-8, 200)
        assert e.value.status == lib.BD_E_INVALID and "scratch" in str(e.value)
        monkeypatch.delenv("BIDOMAIN_NOALLOC_SCRATCH_BYTES")
        rc, info = lib.bidomain_pcg_solve_noalloc(h, b, x, False, 1e-8, 200)
        assert rc == lib.BD_OK and info["rel_residual_true"] <= 1e-8
    finally:
        lib.bidomain_amg_destroy(h)
