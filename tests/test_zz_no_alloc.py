"""The allocation-free build (``bdg_build_knn_noalloc``, static workspace)
against the allocating one (``bdg_build_knn_ex``) through the C ABI: the same
graph on two calls in a row, the second smaller (the static scratch keeps the
first call's contents), and sizes beyond the static scratch rejected before
anything is enqueued."""
import numpy as np
import pytest

from paper_2102_04656_amd import bdg, datagen

pytestmark = pytest.mark.gpu


def _build_pair(d, n, bits, K, stream):
    import torch
    ai = torch.full((n, K), -3, dtype=torch.int32, device="cuda")
    ad = torch.full((n, K), -3, dtype=torch.int16, device="cuda")
    bi = torch.full((n, K), -5, dtype=torch.int32, device="cuda")
    bd = torch.full((n, K), -5, dtype=torch.int16, device="cuda")
    o = bdg.make_opts(path=bdg.PATH_MFMA)
    assert bdg.bdg_build_knn_ex(d, n, bits, K, ai, ad, o, stream) == 0, bdg.last_error()
    assert bdg.bdg_build_knn_noalloc(d, n, bits, K, bi, bd, stream) == 0, bdg.last_error()
    torch.cuda.synchronize()
    return (ai, ad), (bi, bd)


def test_noalloc_matches_the_allocating_build_on_two_calls():
    import torch
    stream = torch.cuda.current_stream()
    for n, bits, K, seed in ((150000, 256, 32, 71), (9000, 512, 100, 72)):
        print(f"[noalloc] n={n} bits={bits} K={K}", flush=True)
        codes = datagen.clustered_codes(n, bits, max(2, n // 500), 0.2, seed=seed)
        d = torch.from_numpy(codes.view(np.int64)).cuda()
        (ai, ad), (bi, bd) = _build_pair(d, n, bits, K, stream)
        assert torch.equal(ai, bi) and torch.equal(ad, bd), f"n={n}: graphs differ"
        assert int(bi[0, 0]) != -5


def test_noalloc_rejects_inputs_beyond_its_scratch():
    import torch
    n, bits, K = 600000, 512, 16
    fake = torch.empty(1, dtype=torch.int64, device="cuda")
    idx = torch.full((4, K), -9, dtype=torch.int32, device="cuda")
    st = bdg.bdg_build_knn_noalloc(fake, n, bits, K, idx, idx, None)
    assert st == bdg.BDG_EUNSUPPORTED and "static workspace" in bdg.last_error()
    torch.cuda.synchronize()
    assert (idx.cpu().numpy() == -9).all()
    assert bdg.bdg_build_knn_noalloc(fake, 0, bits, K, idx, idx, None) == 0
