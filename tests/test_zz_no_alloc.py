"""ski_sketch_noalloc (the sketch with its scratch in a static device array, no device
allocation in the library) against ski_sketch on the same arguments: bit-exact SA, on two
calls in a row with the second smaller, for the dense sketch with the Hadamard transform
(several slabs of the static scratch), the dense sketch without it, and CSR A.  The
oversize refusal is checked too (host-side, before any device work)."""

import sys

import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ski():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2105_11815_amd as P
    return P


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _reference_SA(ski, A, B, **kw):
    S = ski.Solver()
    S.sketch(A, B, **kw)
    SA = S.get_SA()
    S.close()
    return SA


def _dense_pair(ski, n, d, k, m, s, had, seed):
    rng = np.random.default_rng(n + 7 * d)
    A = rng.standard_normal((n, d))
    A[: n // 5] *= 1e3
    B = rng.standard_normal((n, k))
    At, Bt = dev(A), dev(B)
    out = ski.sketch_noalloc(At, Bt, m=m, s=s, seed=seed, hadamard=had)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = _reference_SA(ski, At, Bt, m=m, s=s, seed=seed, hadamard=had)
    return got, ref


# (n, d, k, m, s): the first call of each pair is the larger
DENSE_PAIRS = [
    ((40000, 300, 2, 520, 3), (3000, 70, 1, 150, 2)),   # n' = 65536: three 112-column slabs
    ((9000, 130, 1, 260, 1), (600, 20, 2, 45, 2)),
]


@pytest.mark.parametrize("big,small", DENSE_PAIRS)
def test_noalloc_dense_hadamard_matches_ski_sketch(ski, big, small):
    for i, (n, d, k, m, s) in enumerate((big, small)):
        _say(f"noalloc dense+H call {i}: n={n} d={d} k={k} m={m} s={s}")
        got, ref = _dense_pair(ski, n, d, k, m, s, True, 4242 + i)
        assert got.shape == (m, d + k)
        np.testing.assert_array_equal(got, ref)


def test_noalloc_dense_plain_matches_ski_sketch(ski):
    for i, (n, d, k, m, s) in enumerate(((20000, 200, 1, 400, 3), (1500, 30, 3, 70, 2))):
        _say(f"noalloc dense call {i}: n={n} d={d} k={k} m={m} s={s}")
        got, ref = _dense_pair(ski, n, d, k, m, s, False, 77 + i)
        np.testing.assert_array_equal(got, ref)


def test_noalloc_csr_matches_ski_sketch(ski):
    for i, (n, d, k, m, s) in enumerate(((30000, 400, 1, 600, 2), (2000, 50, 2, 80, 1))):
        _say(f"noalloc csr call {i}: n={n} d={d} k={k} m={m} s={s}")
        rng = np.random.default_rng(n + d)
        M = sp.random(n, d, density=0.02, format="csr", random_state=n,
                      data_rvs=rng.standard_normal)
        M.sort_indices()
        B = rng.standard_normal((n, k))
        A = ("csr", dev(M.indptr.astype(np.int64), torch.int64),
             dev(M.indices.astype(np.int32), torch.int32), dev(M.data), (n, d))
        Bt = dev(B)
        out = ski.sketch_noalloc(A, Bt, m=m, s=s, seed=900 + i, hadamard=False)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref = _reference_SA(ski, A, Bt, m=m, s=s, seed=900 + i, hadamard=False)
        np.testing.assert_array_equal(got, ref)


def test_noalloc_refuses_oversize_and_keeps_working(ski):
    # n' = 2^20: 16 columns of n' doubles need 128 MiB, above the 64 MiB scratch
    _say("noalloc oversize refusal")
    A = torch.zeros((600000, 4), dtype=torch.float64, device="cuda")
    B = torch.zeros((600000, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(ski.SkiError, match="too large"):
        ski.sketch_noalloc(A, B, m=64, s=1, seed=1, hadamard=True)
    got, ref = _dense_pair(ski, 1000, 12, 1, 40, 2, True, 5)
    np.testing.assert_array_equal(got, ref)
