"""CPU-only checks of the HIP library: it loads, exports every entry point the header declares,
and its host-side logic (Q1 assembly, AMG setup) matches the oracle.  No GPU call is made."""
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import bidomain_cases as bc
from oracle import amg, fem

lib = pytest.importorskip("paper_2311_13914_amd")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "bidomain.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bidomain_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = lib.load()
    declared = _declared_symbols()
    assert len(declared) >= 17
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(lib.exported_symbols()) == declared


def test_default_options_follow_appendix_a():
    o = lib.bidomain_default_opts()
    assert o.threshold == 0.06 and o.prolong_smooths == 1 and o.coarse_eq_limit == 100
    assert o.square_graph_levels == 1 and o.smoother_degree == 2 and o.esteig_iters == 10
    assert (o.cheb_lo, o.cheb_hi) == (0.05, 1.05)
    assert o.galerkin_device == 1 and o.diag_form == 1


def _csr(rp, ci, v, n):
    return sp.csr_matrix((v, ci, rp), shape=(n, n))


@pytest.mark.parametrize("name,dims", [("C1", None), ("ragged", (7, 5, 3)), ("aspect", (12, 12, 3))])
def test_host_assembly_matches_oracle(name, dims):
    c = bc.config_case("C1") if dims is None else bc.make_case(*dims, seed=4)
    ops = fem.assemble_operators(c)
    for which, key in ((lib.BD_MAT_AI, "Ai"), (lib.BD_MAT_AE, "Ae"), (lib.BD_MAT_AELL, "Aell"),
                       (lib.BD_MAT_APAR, "Apar")):
        rp, ci, v, m = lib.bidomain_slab_assemble(c, which)
        A = ops[key]
        assert np.array_equal(rp, A.indptr) and np.array_equal(ci, A.indices)
        assert np.max(np.abs(v - A.data)) <= 1e-14 * np.max(np.abs(A.data))
        np.testing.assert_allclose(m, ops["m"], rtol=1e-15)


def _compare_hierarchies(h_lib, h_or, tol=1e-11):
    info = lib.bidomain_amg_info(h_lib)
    assert info["nlevels"] == h_or.nlevels
    assert info["n"] == [lv.A.shape[0] for lv in h_or.levels]
    for k, lv in enumerate(h_or.levels):
        rp, ci, v, shape = lib.bidomain_amg_export(h_lib, k, 0)
        Al = sp.csr_matrix((v, ci, rp), shape=shape)
        assert abs(Al - lv.A).max() <= tol * abs(lv.A).max(), f"A_{k}"
        if np.isfinite(lv.lam):
            assert info["lam"][k] == pytest.approx(lv.lam, rel=1e-10)
        if lv.P is not None:
            rp, ci, v, shape = lib.bidomain_amg_export(h_lib, k, 1)
            Pl = sp.csr_matrix((v, ci, rp), shape=shape)
            assert abs(Pl - lv.P).max() <= tol * abs(lv.P).max(), f"P_{k}"
            rp, ci, v, shape = lib.bidomain_amg_export(h_lib, k, 2)
            Rl = sp.csr_matrix((v, ci, rp), shape=shape)
            assert abs(Rl - lv.R).max() <= tol * abs(lv.R).max(), f"R_{k}"


@pytest.mark.parametrize("variant", ["sa_ell", "sa_par", "rs_ell", "pmis_ell", "luby_ell", "luby_par"])
@pytest.mark.parametrize("dims", [(16, 16, 8), (24, 20, 10)])
def test_host_setup_matches_oracle(variant, dims):
    c = bc.make_case(*dims, seed=1)
    ops = fem.assemble_operators(c)
    if variant == "sa_ell":
        A, oo, lo = ops["Aell"], amg.AMGOptions(nullspace=True), dict(nullspace=1)
    elif variant == "sa_par":
        A, oo, lo = ops["Apar"], amg.AMGOptions(), dict()
    elif variant == "rs_ell":
        A, oo, lo = ops["Aell"], amg.AMGOptions(coarsening="rs", threshold=0.5, nullspace=True), \
            dict(coarsening=lib.BD_RS, threshold=0.5, nullspace=1)
    elif variant == "pmis_ell":
        A, oo, lo = ops["Aell"], amg.AMGOptions(coarsening="pmis", threshold=0.5, nullspace=True, seed=3), \
            dict(coarsening=lib.BD_PMIS, threshold=0.5, nullspace=1, seed=3)
    elif variant == "luby_ell":
        A, oo, lo = ops["Aell"], amg.AMGOptions(nullspace=True, mis="luby", seed=5), \
            dict(nullspace=1, independent_set=lib.BD_MIS_LUBY, seed=5)
    else:
        A, oo, lo = ops["Apar"], amg.AMGOptions(mis="luby", seed=6, threshold=0.0), \
            dict(independent_set=lib.BD_MIS_LUBY, seed=6, threshold=0.0)
    h_or = amg.setup(A, oo)
    h = lib.bidomain_amg_build_host(A, lib.bidomain_default_opts(**lo))
    try:
        _compare_hierarchies(h, h_or)
    finally:
        lib.bidomain_amg_destroy(h)


def test_host_setup_matches_oracle_on_tiny_meshes():
    for dims in [(2, 2, 1), (3, 3, 2), (4, 4, 2)]:
        c = bc.make_case(*dims, seed=3)
        A = fem.assemble_operators(c)["Aell"]
        h_or = amg.setup(A, amg.AMGOptions(nullspace=True, coarse_eq_limit=4))
        h = lib.bidomain_amg_build_host(A, lib.bidomain_default_opts(nullspace=1, coarse_eq_limit=4))
        try:
            _compare_hierarchies(h, h_or)
        finally:
            lib.bidomain_amg_destroy(h)


def test_malformed_csr_is_rejected():
    c = bc.make_case(3, 3, 2, seed=0)
    A = fem.assemble_operators(c)["Aell"]
    bad = A.copy()
    bad.indices = bad.indices.copy()
    bad.indices[[1, 2]] = bad.indices[[2, 1]]  # unsorted row 0
    with pytest.raises(lib.BidomainError) as e:
        lib.bidomain_amg_build_host(bad)
    assert e.value.status == lib.BD_E_INVALID
    neg = A.copy()
    neg.data = neg.data.copy()
    neg.data[neg.indptr[0]] = -1.0  # row 0, col 0 is the diagonal
    with pytest.raises(lib.BidomainError):
        lib.bidomain_amg_build_host(neg)
    with pytest.raises(lib.BidomainError):
        lib.bidomain_amg_build_host(A, lib.bidomain_default_opts(smoother_degree=0))
    # rows are checked in parallel; the message still names the first bad row
    two = A.copy()
    two.data = two.data.copy()
    two.data[two.indptr[9] + 1] = np.nan                   # row 9: non-finite value
    two.data[two.indptr[4]:two.indptr[5]][two.indices[two.indptr[4]:two.indptr[5]] == 4] = -2.0  # row 4
    with pytest.raises(lib.BidomainError) as e:
        lib.bidomain_amg_build_host(two)
    assert "diagonal must be positive in row 4" in str(e.value)


@pytest.mark.parametrize("field,value", [("ap_t_unit", 0.0), ("ap_k", -1.0), ("ap_v_scale", float("nan")),
                                         ("ap_a", float("inf"))])
def test_invalid_membrane_parameters_are_rejected(field, value):
    from dataclasses import replace
    c = replace(bc.make_case(4, 4, 2, seed=1), **{field: value})
    with pytest.raises(lib.BidomainError) as e:
        lib.bidomain_slab_assemble(c, lib.BD_MAT_AELL)
    assert e.value.status == lib.BD_E_INVALID


@pytest.mark.slow
def test_host_code_under_address_and_undefined_behaviour_sanitizers():
    """The host setup code built with -fsanitize=address,undefined runs its self-check (small and
    ragged slabs, every coarsening, smoother and null-space option) without a sanitizer report."""
    import subprocess
    from paper_2311_13914_amd import build
    exe = build.build_host_check()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="4")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert "host check ok" in res.stdout


@pytest.mark.parametrize("dims", [(3, 1, 1), (8, 6, 3), (13, 7, 4)])
def test_host_ellipsoid_assembly_matches_oracle(dims):
    from oracle import ellipsoid
    c = bc.EllipsoidCase(*dims)
    ops = ellipsoid.assemble_operators(c)
    for which, key in ((lib.BD_MAT_AI, "Ai"), (lib.BD_MAT_AE, "Ae"), (lib.BD_MAT_AELL, "Aell"),
                       (lib.BD_MAT_APAR, "Apar")):
        rp, ci, v, m = lib.bidomain_ellipsoid_assemble(c, which)
        A = ops[key]
        assert np.array_equal(rp, A.indptr) and np.array_equal(ci, A.indices)
        assert np.max(np.abs(v - A.data)) <= 1e-14 * np.max(np.abs(A.data))
        np.testing.assert_allclose(m, ops["m"], rtol=1e-13)


def test_host_ellipsoid_setup_matches_oracle():
    """The SA hierarchy of the periodic mesh (its seam makes the fine level a CSR-stream matrix
    rather than a diagonal-form one)."""
    from oracle import ellipsoid
    c = bc.EllipsoidCase(16, 12, 6)
    A = ellipsoid.assemble_operators(c)["Aell"]
    h_or = amg.setup(A, amg.AMGOptions(nullspace=True))
    h = lib.bidomain_amg_build_host(A, lib.bidomain_default_opts(nullspace=1))
    try:
        _compare_hierarchies(h, h_or)
    finally:
        lib.bidomain_amg_destroy(h)


@pytest.mark.parametrize("change", [dict(n_theta=2), dict(n_phi=0), dict(theta_max=0.4 * np.pi),
                                    dict(phi_min=-0.5 * np.pi), dict(phi_max=-0.4 * np.pi), dict(a1=0.0),
                                    dict(sig_it=-1.0), dict(ap_mu2=0.0), dict(dt=float("nan")),
                                    dict(a1=3.3, a2=0.5, b1=3.3, b2=0.5, c1=6.4, c2=0.6)])
def test_invalid_ellipsoids_are_rejected(change):
    from dataclasses import replace
    c = replace(bc.EllipsoidCase(6, 4, 2), **change)
    with pytest.raises(lib.BidomainError) as e:
        lib.bidomain_ellipsoid_assemble(c, lib.BD_MAT_AELL)
    assert e.value.status == lib.BD_E_INVALID


def test_host_galerkin_product_matches_sparse_algebra():
    """bidomain_galerkin on the host: (R A P + (R A P)^T) / 2 with R = P^T on the full structural
    pattern of the product, against scipy's sparse products."""
    import scipy.sparse as sp
    c = bc.make_case(9, 7, 5, seed=2)
    A = fem.assemble_operators(c)["Aell"]
    h = amg.setup(A, amg.AMGOptions(nullspace=True))
    P = h.levels[0].P
    C = lib.bidomain_galerkin(A, P, on_device=False)
    R = (P.T @ A @ P).tocsr()
    ref = 0.5 * (R + R.T)
    assert abs(C - ref).max() <= 1e-13 * abs(ref).max()
    pat = (abs(P.T) @ abs(A) @ abs(P)).tocsr()
    pat.sort_indices()
    assert np.array_equal(C.indptr, pat.indptr) and np.array_equal(C.indices, pat.indices)
    bad = A.copy()
    bad.data = bad.data.copy()
    bad.data[bad.indptr[0]] = -1.0      # row 0's diagonal
    with pytest.raises(lib.BidomainError):
        lib.bidomain_galerkin(bad, P, on_device=False)
    assert lib.bidomain_galerkin(A, sp.csr_matrix(P.shape), on_device=False).nnz == 0
