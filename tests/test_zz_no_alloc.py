"""The allocation-free heat bath (su2_heatbath_noalloc, for callers that
cannot allocate) against the handle's su2_heatbath through the C ABI: the
same links, bit for bit, from the same starting links, coupling, seed and
sweep counter, on calls in a row whose second input is smaller (the shared
device scratch keeps the previous call's contents)."""
import numpy as np
import pytest

from tests import inputs

pytestmark = pytest.mark.gpu


def test_noalloc_heatbath_matches_handle():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1010_4834_amd import su2
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    err = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    cases = (((8, 6, 4, 10), su2.F32, 2.4, 3, 9), ((4, 4, 2, 6), su2.F32, 2.7, 2, 5),
             ((6, 4, 4, 8), su2.F64, 2.3, 2, 4), ((4, 2, 2, 4), su2.F64, 1.9, 1, 8))
    for k, (dims, prec, beta, n, seed) in enumerate(cases):
        print(f"noalloc case {k}: dims {dims} prec {prec} beta {beta} sweeps {n}", flush=True)
        lat = su2.Lattice(dims, start=su2.COLD, prec=prec)
        lat.set_links(inputs.random_config(dims, 71 + k))
        lat.sweep = 3 * k                                   # a non-zero counter too
        torch.cuda.synchronize()
        buf = lat._buf.clone()                               # the same native links
        torch.cuda.synchronize()
        lat.heatbath(beta, n, seed)
        err.fill_(7)
        torch.cuda.synchronize()
        su2.su2_heatbath_noalloc(buf.data_ptr(), dims, prec, beta, n, seed, 3 * k, err.data_ptr(),
                                 stream.cuda_stream)
        stream.synchronize()
        assert int(err.item()) == 0
        assert torch.equal(buf, lat._buf), k
        assert lat.sweep == 3 * k + n
        lat.close()
    # beyond the scratch limit of 2^27 sites: refused before any launch
    big = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(su2.SU2Error) as e:
        su2.su2_heatbath_noalloc(big.data_ptr(), (256, 256, 256, 16), su2.F32, 2.3, 1, 1)
    assert e.value.status == su2.EINVAL
