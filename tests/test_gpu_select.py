"""Ordered compaction (nphc_select) against numpy: random codes of several
lengths (ragged last tiles, empty and single-item lists), one-workgroup and
multi-workgroup forms."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [0, 1, 255, 256, 257, 70001, 262144, 1048575])
@pytest.mark.parametrize("with_ws", [False, True])
def test_select_matches_numpy(n, with_ws):
    import torch
    from paper_1104_5497_amd import _lib as L
    rng = np.random.default_rng(n + 7)
    code = rng.integers(-2, 70, size=max(n, 1)).astype(np.int32)[:n]
    mask = (1 << 10) | (1 << 13) | (1 << 63)
    dev = "cuda"
    c = torch.from_numpy(code.copy() if n else np.zeros(1, np.int32)).to(dev)
    out = torch.full((max(n, 1),), -1, dtype=torch.int64, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = torch.zeros(max(8, int(L.lib().nphc_select_workspace_size(n))), dtype=torch.uint8,
                     device=dev)
    p = lambda x: ctypes.c_void_p(x.data_ptr())
    print(f"select n={n} ws={with_ws}", flush=True)
    L.check(L.lib().nphc_select(p(c), n, mask, p(out), p(cnt), p(ws) if with_ws else None,
                                ws.numel() if with_ws else 0,
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
            "nphc_select")
    torch.cuda.synchronize()
    want = np.nonzero(np.isin(code, [10, 13, 63]))[0]
    k = int(cnt.item())
    assert k == want.size
    assert np.array_equal(out[:k].cpu().numpy(), want)


@pytest.mark.parametrize("n,k,dev_len", [(1000, 0, None), (1000, 1, None), (5000, 257, None),
                                         (262144, 70001, None), (262144, 70001, 123),
                                         (262144, 70001, 0), (262144, 70001, -5),
                                         (262144, 70001, 10 ** 9)])
@pytest.mark.parametrize("with_ws", [False, True])
def test_select_list_matches_numpy(n, k, dev_len, with_ws):
    """nphc_select_list: a sorted random list of k of n items, its length read
    on the device (clamped to [0, k]) when dev_len is given; the matches in
    list order."""
    import torch
    from paper_1104_5497_amd import _lib as L
    rng = np.random.default_rng(n + k + 3)
    code = rng.integers(-2, 70, size=n).astype(np.int32)
    ids = np.sort(rng.choice(n, k, replace=False)).astype(np.int64)
    mask = (1 << 10) | (1 << 13) | (1 << 63)
    dev = "cuda"
    c = torch.from_numpy(code).to(dev)
    li = torch.from_numpy(ids if k else np.zeros(1, np.int64)).to(dev)
    out = torch.full((max(k, 1),), -1, dtype=torch.int64, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    dl = torch.tensor([dev_len if dev_len is not None else 0], dtype=torch.int64, device=dev)
    ws = torch.zeros(max(8, int(L.lib().nphc_select_workspace_size(k))), dtype=torch.uint8,
                     device=dev)
    p = lambda x: ctypes.c_void_p(x.data_ptr())
    print(f"select_list n={n} k={k} dev_len={dev_len} ws={with_ws}", flush=True)
    L.check(L.lib().nphc_select_list(p(c), p(li), k, p(dl) if dev_len is not None else None, mask,
                                     p(out), p(cnt), p(ws) if with_ws else None,
                                     ws.numel() if with_ws else 0,
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
            "nphc_select_list")
    torch.cuda.synchronize()
    length = k if dev_len is None else min(max(dev_len, 0), k)
    sub = ids[:length]
    want = sub[np.isin(code[sub], [10, 13, 63])]
    got = int(cnt.item())
    assert got == want.size
    assert np.array_equal(out[:got].cpu().numpy(), want)
