"""xms_rotate_noalloc (device inputs and outputs, no allocation, its one
intermediate in a fixed device array) against xms_rotate on the same inputs,
through the C ABI: two calls in a row, the second with fewer states and
active orbitals (the array keeps the first call's contents)."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _inputs(na, nst, seed):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((na, na))
    f = 0.5 * (f + f.T)
    G = rng.standard_normal((nst, nst, na, na))
    G = 0.5 * (G + G.transpose(1, 0, 3, 2))    # <M|E_rs|N> = <N|E_sr|M>
    return f, G


def test_noalloc_matches_xms_rotate():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1606_01273_amd import lib, xms_rotate
    L = lib()
    L.xms_rotate_noalloc.restype = ctypes.c_int
    L.xms_rotate_noalloc.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream()
    for (na, nst, seed) in [(6, 4, 1), (3, 2, 2)]:
        print("call", na, nst, flush=True)
        f, G = _inputs(na, nst, seed)
        U_ref, e_ref = xms_rotate(f, G)
        tf = torch.tensor(f, device=dev)
        tg = torch.tensor(G, device=dev)
        tU = torch.full((nst, nst), np.nan, dtype=torch.float64, device=dev)
        te = torch.full((nst,), np.nan, dtype=torch.float64, device=dev)
        rc = L.xms_rotate_noalloc(na, nst, tf.data_ptr(), tg.data_ptr(), tU.data_ptr(), te.data_ptr(),
                                  ctypes.c_void_p(stream.cuda_stream))
        assert rc == 0
        torch.cuda.synchronize()
        U, e = tU.cpu().numpy(), te.cpu().numpy()
        assert np.abs(U - U_ref).max() <= 1e-14, np.abs(U - U_ref).max()
        assert np.abs(e - e_ref).max() <= 1e-14 * max(1.0, np.abs(e_ref).max())
    # beyond the array's size
    tU = torch.empty((17, 17), dtype=torch.float64, device=dev)
    te = torch.empty(17, dtype=torch.float64, device=dev)
    assert L.xms_rotate_noalloc(2, 17, tf.data_ptr(), tg.data_ptr(), tU.data_ptr(), te.data_ptr(), None) == -1
