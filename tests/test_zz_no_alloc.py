"""The perceptron forward pass without a workspace
(scc_mlp_forward_noalloc, library-owned device scratch) against the
workspace version scc_mlp_forward on the same inputs: identical outputs on
two calls in a row, the second with a smaller batch (the scratch keeps the
first call's contents, which must not leak into the second), plus the size
limit of the scratch."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_forward_without_workspace_matches_forward():
    import torch
    from paper_2403_01007_amd.binding import Mlp, MlpDims, load_library
    nin, nh, nout = 36, 256, 131
    rng = np.random.Generator(np.random.PCG64(11))
    count = nh * nin + nh + nh * nh + nh + nout * nh + nout
    params = rng.normal(0, 0.1, size=count).astype(np.float32)
    net = Mlp(nin, nh, nout, params)
    print("[mlp forward without workspace: batches 700 then 37]", flush=True)
    for n in (700, 37):
        X = rng.normal(0, 0.05, size=(n, nin)).astype(np.float32)
        a = net.forward_noalloc(X).cpu().numpy()
        b = net.forward(X).cpu().numpy()
        assert a.shape == (n, nout)
        assert np.array_equal(a, b)
    # beyond the scratch: 2 * n * nhidden > 2^20 floats is refused before any work
    lib = load_library()
    d = MlpDims(nin, nh, nout)
    n = (1 << 20) // (2 * nh) + 1
    X = torch.zeros((n, nin), dtype=torch.float32, device="cuda:0")
    Y = torch.zeros((n, nout), dtype=torch.float32, device="cuda:0")
    rc = lib.scc_mlp_forward_noalloc(ctypes.byref(d), ctypes.c_void_p(net.params.data_ptr()), n,
                                     ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()), None)
    assert rc == -7
    assert float(Y.abs().max()) == 0.0
