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
