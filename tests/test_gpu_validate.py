"""GPU check of the canonical-CSR validator (hp_validate_csr)."""
import pytest
import torch

import synth
from tests._gpu import mixed_csr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_20776_amd import hipperm
    return hipperm


def test_validator(hp):
    h = hp.handle(0)
    A = mixed_csr(41, 200, 300, [0, 1, 5, 40, 120])
    h.validate(A)
    h.validate(synth.workload_er_small(device="cuda")["A"])
    bad = synth.CSR(A.nrows, A.ncols, A.rowptr, A.col.clone(), A.val)
    rp = A.rowptr.cpu()
    r = int(torch.nonzero(rp[1:] - rp[:-1] >= 5)[0])
    s = int(rp[r])
    bad.col[s], bad.col[s + 1] = A.col[s + 1], A.col[s]       # unsorted row
    with pytest.raises(hp.HPError) as e:
        h.validate(bad)
    assert e.value.name == "HP_ERR_NOT_CANONICAL"
    bad2 = synth.CSR(A.nrows, A.ncols, A.rowptr, A.col.clone(), A.val)
    bad2.col[-1] = A.ncols                                      # column out of range
    with pytest.raises(hp.HPError) as e:
        h.validate(bad2)
    assert e.value.name == "HP_ERR_INDEX_RANGE"


def test_plans_validate_inputs_when_switched_on(hp):
    """With validation on, every CSR plan checks its inputs first: a
    non-canonical A (or B) is refused before anything else runs, and
    canonical inputs give the same results as with validation off."""
    import numpy as np
    from tests._gpu import assert_same, np_csr
    h = hp.Handle(0)
    A = mixed_csr(43, 300, 250, [0, 1, 5, 40, 120], torch.int64, torch.float64)
    p = synth.randperm(44, A.nrows, "cuda")
    q = synth.randperm(45, A.ncols, "cuda")
    I = synth.subset(46, A.nrows, 90, repeat_frac=0.1, device="cuda")
    J = synth.subset(47, A.ncols, 70, repeat_frac=0.1, device="cuda")
    Ia = synth.subset(48, A.nrows, 30, device="cuda")
    Ja = synth.subset(49, A.ncols, 20, device="cuda")
    B = synth.bernoulli_block(30, 20, 0.2, 50, "vB", ptr_dtype=torch.int64, val_dtype=torch.float64, device="cuda")
    ref = [np_csr(h.permute(A, p, q)), np_csr(h.spref(A, I, J)), np_csr(h.spasgn(A, B, Ia, Ja, "plus")),
           np_csr(h.spasgn_permute(A, B, Ia, Ja, p, q, "second"))]
    h.set_validate(True)
    got = [np_csr(h.permute(A, p, q)), np_csr(h.spref(A, I, J)), np_csr(h.spasgn(A, B, Ia, Ja, "plus")),
           np_csr(h.spasgn_permute(A, B, Ia, Ja, p, q, "second"))]
    for k in range(4):
        assert_same(got[k], ref[k], f"call {k} with validation")
    rp = A.rowptr.cpu().numpy()
    r = int(np.nonzero(np.diff(rp) >= 5)[0][0])
    s = int(rp[r])
    bad = synth.CSR(A.nrows, A.ncols, A.rowptr, A.col.clone(), A.val)
    bad.col[s], bad.col[s + 1] = A.col[s + 1], A.col[s]
    for call in (lambda: h.permute(bad, p, q), lambda: h.spref(bad, I, J),
                 lambda: h.spasgn(bad, B, Ia, Ja), lambda: h.spasgn_permute(bad, B, Ia, Ja, p, q)):
        with pytest.raises(hp.HPError) as e:
            call()
        assert e.value.name == "HP_ERR_NOT_CANONICAL"
    badB = synth.CSR(B.nrows, B.ncols, B.rowptr, B.col.clone(), B.val)
    badB.col[-1] = B.ncols + 3
    with pytest.raises(hp.HPError) as e:
        h.spasgn(A, badB, Ia, Ja)
    assert e.value.name == "HP_ERR_INDEX_RANGE"
    h.set_validate(False)
    assert_same(np_csr(h.permute(A, p, q)), ref[0], "validation off again")
    h.close()
