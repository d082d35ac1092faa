"""The seeded input generators produce what they claim (CPU only)."""

import numpy as np
import pytest

import synth


def test_householder_known_has_the_spectrum():
    torch = pytest.importorskip("torch")
    for m, n in [(300, 60), (40, 90), (1, 5), (7, 1)]:
        s = synth.spectrum_geometric(0.95, min(m, n))
        A = synth.householder_known_torch(m, n, s, seed=3, device="cpu")
        assert A.dtype == torch.float32 and tuple(A.shape) == (m, n)
        sv = np.linalg.svd(A.double().numpy(), compute_uv=False)
        assert np.max(np.abs(sv - s) / s) < 5e-7  # FP32 rounding of an exact construction
    # no reflections: the plain diagonal; reflections make it dense
    s = synth.spectrum_geometric(0.9, 8)
    D = synth.householder_known_torch(10, 8, s, seed=1, device="cpu", reflectors=0).numpy()
    assert np.array_equal(D[:8, :8], np.diag(s).astype(np.float32)) and not D[8:].any()
    H = synth.householder_known_torch(10, 8, s, seed=1, device="cpu").numpy()
    assert np.count_nonzero(H) == H.size


def test_householder_known_is_seeded():
    pytest.importorskip("torch")
    s = synth.spectrum_geometric(0.95, 20)
    a = synth.householder_known_torch(50, 20, s, seed=4, device="cpu").numpy()
    b = synth.householder_known_torch(50, 20, s, seed=4, device="cpu").numpy()
    c = synth.householder_known_torch(50, 20, s, seed=5, device="cpu").numpy()
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_request_stream_shapes_and_rate():
    reqs = synth.request_stream(4000, 200.0, seed=1)
    t = np.array([r.t for r in reqs])
    assert t[0] == 0 and np.all(np.diff(t) >= 0)
    assert abs(np.mean(np.diff(t)) - 1 / 200.0) < 0.1 / 200.0
    ms = np.array([r.m for r in reqs]); ns = np.array([r.n for r in reqs])
    assert ms.min() >= 1024 and ms.max() <= 65536 and ns.min() >= 128 and ns.max() <= 4096
    assert {r.k for r in reqs} <= {8, 16, 32, 64}
    # log-uniform: the median of log m sits mid-range
    assert abs(np.median(np.log(ms)) - (np.log(1024) + np.log(65536)) / 2) < 0.15


def test_spiked_rows_torch_row_ranges_and_spikes():
    torch = pytest.importorskip("torch")
    a = synth.spiked_rows_torch(20000, 48, 3, 1, 0, 20000, "cpu")
    b = synth.spiked_rows_torch(20000, 48, 3, 1, 16380, 10, "cpu")  # crosses a 2^14-row block edge
    assert torch.equal(a[16380:16390], b)
    sv = np.linalg.svd(a.double().numpy(), compute_uv=False)
    theta = 50 * np.sqrt(20000) * 0.9 ** np.arange(3)
    # spikes far above the noise bulk (~sqrt(m) + sqrt(n)); x is orthonormal to O(1/sqrt(m))
    assert np.all(np.abs(sv[:3] - theta) / theta < 0.05) and sv[3] < 2 * (np.sqrt(20000) + np.sqrt(48))


def test_csr_uniform_torch_is_valid_csr():
    torch = pytest.importorskip("torch")
    rp, col, val = synth.csr_uniform_torch(3000, 7000, 0.002, 4, "cpu")
    assert rp.dtype == torch.int64 and col.dtype == torch.int32 and val.dtype == torch.float32
    assert int(rp[0]) == 0 and bool(torch.all(rp[1:] >= rp[:-1])) and int(rp[-1]) == col.numel() == val.numel()
    assert int(col.min()) >= 0 and int(col.max()) < 7000
    assert abs(col.numel() / (3000 * 7000 * 0.002) - 1) < 0.05
    rp2, col2, _ = synth.csr_uniform_torch(3000, 7000, 0.002, 4, "cpu")
    assert torch.equal(rp, rp2) and torch.equal(col, col2)
