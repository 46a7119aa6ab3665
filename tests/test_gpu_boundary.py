"""The C ABI's handle state on the device: the encoder's workspace query, sticky device
faults per handle, and stream-ordered dictionary uploads that leave launches in flight
on their own dictionary (the calls of Sec. II-B's problem statement: patches, M atoms,
K, R angles)."""
import numpy as np
import pytest
import torch

from paper_1806_04374_amd import rsc
from paper_1806_04374_amd import workloads as wl

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def _dict(M, seed):
    return wl.draw_dictionary(M, 55, seed=seed).astype(np.float32)


def _xhat(P, seed):
    g = torch.Generator().manual_seed(seed)
    return torch.randn((P, 55), generator=g, dtype=torch.float32).to(DEV)


def _alone(D, R, xh, K):
    """Codes of a fresh handle holding only D (the same kernels and tables)."""
    h = rsc.rsc_create(11, 5, 5)
    rsc.rsc_set_dictionary(h, D, R)
    out = rsc.rsc_omp_encode(h, xh, K)
    torch.cuda.synchronize()
    res = [t.cpu() for t in out[:3]]
    h.close()
    return res


def _same(a, b):
    return all(torch.equal(x.cpu(), y) for x, y in zip(a[:3], b))


def test_encode_workspace_is_zero():
    h = rsc.rsc_create(11, 5, 5)
    rsc.rsc_set_dictionary(h, _dict(16, 1), 32)
    for P, K in ((0, 1), (1, 4), (10**6, 8)):
        assert rsc.rsc_encode_workspace_size(h, P, K) == 0
    with pytest.raises(rsc.RscError):
        rsc.rsc_encode_workspace_size(h, 10, 9)
    h.close()


def test_sticky_fault_is_per_handle():
    h1, h2 = rsc.rsc_create(11, 5, 5), rsc.rsc_create(11, 5, 5)
    D = _dict(16, 2)
    for h in (h1, h2):
        rsc.rsc_set_dictionary(h, D, 32)
    xh = _xhat(1000, 3)
    ref = rsc.rsc_omp_encode(h1, xh, 2)
    rsc.rsc_sync(h1)
    rsc.rsc_set_fault(h1, "planted fault")
    for call in (lambda: rsc.rsc_omp_encode(h1, xh, 2), lambda: rsc.rsc_project(h1, torch.zeros((4, 11, 11), device=DEV)),
                 lambda: rsc.rsc_set_dictionary(h1, D, 32), lambda: rsc.rsc_sync(h1)):
        with pytest.raises(rsc.RscError) as e:
            call()
        assert e.value.status == rsc.RSC_E_DEVICE and "planted fault" in str(e.value)
    assert "planted fault" in rsc.rsc_last_error(h1)
    rsc.rsc_set_fault(h1, "second")                       # the first message stays
    with pytest.raises(rsc.RscError, match="planted fault"):
        rsc.rsc_sync(h1)
    # the other handle is untouched
    out = rsc.rsc_omp_encode(h2, xh, 2)
    rsc.rsc_sync(h2)
    rsc.rsc_sync(None)
    assert all(torch.equal(a, b) for a, b in zip(out[:3], ref[:3]))
    h1.close()
    h2.close()


def test_dictionary_swap_while_another_stream_encodes():
    """Encodes in flight keep the dictionary they were launched with; launches after the
    upload returns (on either stream) use the new one; an upload that overwrites the
    older copy waits for its readers."""
    P, K, R = 1_000_000, 4, 64
    D1, D2, D3, D4 = (_dict(64, s) for s in (11, 12, 13, 14))
    xh = _xhat(P, 5)
    ref = {i: _alone(D, R, xh, K) for i, D in enumerate((D1, D2, D3, D4), 1)}
    assert not _same(ref[1], ref[2])
    h = rsc.rsc_create(11, 5, 5)
    a, b = torch.cuda.Stream(DEV), torch.cuda.Stream(DEV)
    rsc.rsc_set_dictionary(h, D1, R, stream=a)
    torch.cuda.synchronize()
    e1 = rsc.rsc_omp_encode(h, xh, K, stream=a)           # in flight (milliseconds)
    rsc.rsc_set_dictionary(h, D2, R, stream=b)             # fills the other copy
    e2 = rsc.rsc_omp_encode(h, xh, K, stream=a)            # after the upload: D2
    e3 = rsc.rsc_omp_encode(h, xh, K, stream=b)            # D2
    rsc.rsc_set_dictionary(h, D3, R, stream=b)             # overwrites D1's copy after e1
    e4 = rsc.rsc_omp_encode(h, xh, K, stream=a)            # D3
    rsc.rsc_set_dictionary(h, D4, R, stream=b)             # overwrites D2's copy after e2, e3
    e5 = rsc.rsc_omp_encode(h, xh, K, stream=b)            # D4
    torch.cuda.synchronize()
    rsc.rsc_sync(h, a)
    assert _same(e1, ref[1])
    assert _same(e2, ref[2]) and _same(e3, ref[2])
    assert _same(e4, ref[3])
    assert _same(e5, ref[4])
    h.close()


def test_refused_upload_keeps_the_dictionary():
    h = rsc.rsc_create(11, 5, 5)
    D = _dict(16, 21)
    rsc.rsc_set_dictionary(h, D, 32)
    xh = _xhat(2000, 22)
    ref = rsc.rsc_omp_encode(h, xh, 2)
    bad = D.copy()
    bad[3] *= 2.0
    with pytest.raises(rsc.RscError) as e:
        rsc.rsc_set_dictionary(h, bad, 32)                 # rows not unit norm
    assert e.value.status == rsc.RSC_E_INVALID
    with pytest.raises(rsc.RscError) as e:
        rsc.rsc_set_dictionary(h, D, 129)                  # R out of range
    assert e.value.status == rsc.RSC_E_INVALID
    out = rsc.rsc_omp_encode(h, xh, 2)
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(out[:3], ref[:3]))
    # a smaller dictionary, then the first again: tables of either size in either copy
    rsc.rsc_set_dictionary(h, _dict(4, 23), 8)
    rsc.rsc_omp_encode(h, xh, 2)
    rsc.rsc_set_dictionary(h, D, 32)
    out = rsc.rsc_omp_encode(h, xh, 2)
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(out[:3], ref[:3]))
    h.close()


def test_handles_used_from_two_threads_at_once():
    """The library is safe across handles: two threads, each with its own handle, dictionary
    and stream, project and encode at the same time (the binding releases the interpreter lock
    during the calls); every result equals the codes its handle gives when used alone."""
    import threading
    K, R = 4, 64
    cases = [(_dict(64, 31), _xhat(20000, 32)), (_dict(48, 33), _xhat(15000, 34))]
    want = [_alone(D, R, xh, K) for D, xh in cases]
    errors = []

    def work(i):
        try:
            D, xh = cases[i]
            st = torch.cuda.Stream()
            h = rsc.rsc_create(11, 5, 5)
            rsc.rsc_set_dictionary(h, D, R, stream=st)
            for _ in range(5):
                with torch.cuda.stream(st):
                    out = rsc.rsc_omp_encode(h, xh, K, stream=st)
                st.synchronize()
                if not _same(out, want[i]):
                    errors.append(f"thread {i}: codes differ")
            rsc.rsc_sync(h, st)
            h.close()
        except Exception as e:       # noqa: BLE001 -- collected and asserted below
            errors.append(f"thread {i}: {e!r}")

    threads = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(120)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors
