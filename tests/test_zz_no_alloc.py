"""The no-allocation expectation entry point against the allocating one:
same kernels and plan on the same state, so the terms agree to FP64 rounding
of the fixed-order sums (the grids are the same size on MI355X, making them
identical there).  Two calls in a row, the second with a smaller state and
fewer terms (the array keeps the first call's contents), and the size limit."""
import numpy as np
import pytest

import qsynth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    import torch

    from paper_2509_04955_amd import qsim

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    qsim.lib()
    return qsim


@pytest.mark.parametrize("dtype", [0, 1])
def test_noalloc_matches_allocating_entry_point(Q, dtype):
    for n, n_terms, seed in ((22, 300, 1), (16, 40, 2)):
        psi = qsynth.random_state(n, seed=seed)
        ham = qsynth.random_pauli_sum(n, n_terms, seed=(seed, 5))
        s = Q.State(n, dtype)
        s.load(psi)
        E1, t1 = Q.qs_expect_pauli_sum(s.handle, ham.x, ham.z, ham.coeff, with_terms=True)
        E2, t2 = Q.qs_expect_pauli_sum_noalloc(s.handle, ham.x, ham.z, ham.coeff, with_terms=True)
        s.close()
        assert np.max(np.abs(t1 - t2)) <= 1e-14, (n, np.max(np.abs(t1 - t2)))
        assert abs(E1 - E2) <= 1e-12
        assert np.count_nonzero(np.abs(t1) > 1e-6) > 0


def test_noalloc_rejects_more_terms_than_it_holds(Q):
    n = 10
    ham = qsynth.random_pauli_sum(n, 2049, seed=(3, 3))
    s = Q.State(n, Q.QS_C128)
    with pytest.raises(Q.QsimError) as ei:
        Q.qs_expect_pauli_sum_noalloc(s.handle, ham.x, ham.z, ham.coeff)
    assert ei.value.status == Q.QS_ERANGE
    # the limit itself is accepted
    E = Q.qs_expect_pauli_sum_noalloc(s.handle, ham.x[:2048], ham.z[:2048], ham.coeff[:2048])
    E_ref = Q.qs_expect_pauli_sum(s.handle, ham.x[:2048], ham.z[:2048], ham.coeff[:2048])
    s.close()
    assert abs(E - E_ref) <= 1e-12
