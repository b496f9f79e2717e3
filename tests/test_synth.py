"""The shared input generators: the counter-based stream is SplitMix64 by its
published definition, and each workload has the structure it claims."""
import torch

import synth


def test_splitmix64_published_first_output():
    # SplitMix64 seeded with 0: first output 0xE220A8397B1DCDAF (reference implementation)
    assert synth.splitmix64_ref(0, 1)[0] == 0xE220A8397B1DCDAF


def test_tensor_stream_equals_reference_sequence():
    for key in (0, 1, 0xDEADBEEF, 2 ** 63 + 5):
        ref = synth.splitmix64_ref(key, 50)
        got = synth.draws(key, 50)
        assert [x & synth.MASK64 for x in got.tolist()] == ref


def test_randperm_and_values():
    p = synth.randperm(123, 1000)
    assert torch.equal(torch.sort(p).values, torch.arange(1000, dtype=torch.int32))
    v = synth.values(5, 10000, torch.float64)
    assert float(v.min()) > 0 and float(v.max()) <= 1
    v32 = synth.values(5, 10000, torch.float32)
    assert v32.dtype == torch.float32 and float(v32.min()) > 0


def test_grid_structure():
    A = synth.grid5(5, 7)
    assert A.nnz == 4 * 5 * 7 - 2 * 5 - 2 * 7
    rp = A.rowptr.tolist()
    for r in range(35):
        cols = A.col[rp[r]:rp[r + 1]].tolist()
        assert cols == sorted(set(cols))
        for c in cols:
            assert abs(c - r) in (1, 7) and c != r


def test_rmat_canonical_and_symmetric():
    A = synth.rmat(10, 8, seed=3, symmetric=True)
    rp, c = A.rowptr.long(), A.col.long()
    for r in range(A.nrows):
        seg = c[rp[r]:rp[r + 1]]
        assert torch.all(seg[1:] > seg[:-1])
    rows = torch.repeat_interleave(torch.arange(A.nrows), rp[1:] - rp[:-1])
    fw = set(zip(rows.tolist(), c.tolist()))
    assert all((b, a) in fw for (a, b) in fw)
    deg = (rp[1:] - rp[:-1])
    assert int(deg[:8].sum()) > int(deg[-8:].sum())     # hubs at low ids


def test_subset_repeats():
    I = synth.subset(9, 1000, 400, sort=False, repeat_frac=0.01)
    assert I.numel() == 400
    assert len(set(I.tolist())) == 400 - 4
    S = synth.subset(9, 1000, 250, sort=True)
    assert S.tolist() == sorted(set(S.tolist()))


def test_workloads_small():
    w = synth.workload_er_small(n=512)
    assert w["A"].nrows == 512 and w["I"].numel() == 128
    g = synth.workload_grid(side=32)
    k = int(0.1 * 32 * 32)
    assert g["B"].nrows == k and g["B"].ncols == k
    assert g["I"].tolist() == list(range(int(g["I"][0]), int(g["I"][0]) + k))
