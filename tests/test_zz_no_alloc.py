"""The allocation-free field S(k) entry point (fsc_field_sk_noalloc) against the
allocating one (fsc_field_sk) and the oracle, through the C ABI.

Two calls in a row share the library's fixed-size device scratch, the second
on a smaller input; a third call repeats the first, so a stale accumulator or
twiddle table left by an earlier call would show.  Both entry points run the
same kernels in the same order; their results may differ only in the order of
the FP64 atomic additions of the binning (1e-12 relative).  Against the oracle
the FP32 FFT of fields near 1 (the mean is transformed too) gives per-shell
errors up to about 1e-4 (a CPU single-precision FFT of the same fields: 8e-5);
the bound is 5e-4.
"""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

fsc = pytest.importorskip("paper_2212_07848_amd")
torch = pytest.importorskip("torch")


def _fields(batch, n, seed):
    rng = np.random.default_rng(seed)
    f = 1.0 + 0.1 * rng.normal(size=(batch, n, n))
    return f.astype(np.float32)


def _check_against_allocating_and_oracle(host, n):
    batch = host.shape[0]
    dev = torch.from_numpy(host).cuda()
    torch.cuda.synchronize()
    print(f"field S(k): batch {batch}, {n}x{n}, no-alloc and allocating entry points", flush=True)
    s_na, l_na = fsc.field_sk(dev, batch, n, noalloc=True)
    s_al, l_al = fsc.field_sk(dev, batch, n, noalloc=False)
    assert np.allclose(s_na, s_al, rtol=1e-12, atol=0.0)
    assert np.allclose(l_na, l_al, rtol=1e-12, atol=0.0)
    for b in range(batch):
        f64 = host[b].astype(np.float64)
        ref = O.shell_means(f64)
        nz = ref > 0
        assert np.all(np.abs(s_na[b] - ref) <= 5e-4 * ref + 1e-6 * ref[nz].mean())
        assert l_na[b] == pytest.approx(O.domain_length(f64), rel=5e-4)
    return s_na, l_na


def test_noalloc_field_sk_matches_allocating_entry_point_twice():
    first = _fields(3, 256, seed=1)
    s1, l1 = _check_against_allocating_and_oracle(first, 256)
    # second call, smaller input, same scratch
    _check_against_allocating_and_oracle(_fields(2, 64, seed=2), 64)
    # the first input again: nothing of the previous calls leaks through
    s3, l3 = _check_against_allocating_and_oracle(first, 256)
    assert np.allclose(s3, s1, rtol=1e-12, atol=0.0) and np.allclose(l3, l1, rtol=1e-12, atol=0.0)
    # a ragged (non power-of-two) side runs the DFT path through the same scratch
    _check_against_allocating_and_oracle(_fields(1, 96, seed=3), 96)


def test_noalloc_field_sk_rejects_fields_beyond_its_scratch():
    import ctypes
    small = torch.zeros(16, dtype=torch.float32, device="cuda")
    n = 2048
    c = ctypes.c_int()
    fsc.lib().fsc_field_nbins(n, ctypes.byref(c))
    nb = c.value
    shells = np.zeros(nb)
    L = np.zeros(1)
    rc = fsc.lib().fsc_field_sk_noalloc(ctypes.c_void_p(small.data_ptr()), 1, n, n, None,
                                        shells.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        L.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nb)
    assert rc == -8
    assert fsc.lib().fsc_strerror(rc).decode().startswith("input larger")
