"""The allocation-free compaction entry point (cgsr_compact_gaussians_noalloc)
against the allocating one (cgsr_compact_gaussians), through the C ABI: the
same Gaussians, extra arrays and count, byte for byte, on two calls in a row
(the second smaller, so it reads counters the first left behind in the
library's fixed scratch), and both against the oracle's compaction."""
import sys

import numpy as np
import pytest

from oracle import management as M
from paper_2403_16095_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def t32(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def compact_both(B, R, sc, keep, extra):
    """Both entry points on the same inputs; returns their outputs and counts."""
    n = sc["means"].shape[0]
    src = {k: t32(v) for k, v in sc.items()}
    keep_t = torch.from_numpy(keep).cuda()
    ex_src = [t32(e) for e in extra]
    widths = [int(e.shape[1]) if e.ndim == 2 else 1 for e in extra]
    res = []
    for fn in (B.cgsr_compact_gaussians, B.cgsr_compact_gaussians_noalloc):
        dst = R.empty_like_set(src, n)
        for v in dst.values():
            v.fill_(float("nan"))
        ex_dst = [torch.full_like(e, float("nan")) for e in ex_src]
        m = fn(n, keep_t.data_ptr(), R.arrays_struct(src), R.arrays_struct(dst), [e.data_ptr() for e in ex_src],
               [e.data_ptr() for e in ex_dst], widths, torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        res.append((m, {k: v[:m].cpu().numpy() for k, v in dst.items()}, [e[:m].cpu().numpy() for e in ex_dst]))
    return res


@pytest.mark.parametrize("sh", [False, True])
def test_noalloc_compaction_equals_allocating_one(sh):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_16095_amd import binding as B
    from paper_2403_16095_amd import rasterizer as R
    for call, (n, p_keep) in enumerate(((300_007, 0.7), (5_003, 0.4))):
        say(f"case: no-alloc compaction call {call + 1}: {n} Gaussians, keep {p_keep}, sh {sh}")
        rng = np.random.default_rng(100 + call + 10 * sh)
        sc = synth.uniform_box_scene(11 + call, n)
        if sh:
            sc["sh"] = synth.sh_coefficients(12 + call, n, 2)
            del sc["rgb"]
        keep = (rng.random(n) < p_keep).astype(np.uint8)
        extra = [rng.standard_normal((n, 4)).astype(np.float32), rng.standard_normal(n).astype(np.float32)]
        (m_a, out_a, ex_a), (m_b, out_b, ex_b) = compact_both(B, R, sc, keep, extra)
        assert m_a == m_b == int(keep.sum())
        for k in out_a:
            assert out_a[k].tobytes() == out_b[k].tobytes(), k
        for a, b in zip(ex_a, ex_b):
            assert a.tobytes() == b.tobytes()
        ref = M.compact(sc, keep)
        for k in sc:
            np.testing.assert_array_equal(out_b[k], ref[k], err_msg=k)
        kb = keep.astype(bool)
        for e, b in zip(extra, ex_b):
            np.testing.assert_array_equal(b, e[kb])


def test_noalloc_compaction_limits():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_16095_amd import binding as B
    from paper_2403_16095_amd import rasterizer as R
    say("case: no-alloc compaction of 0 Gaussians and one over the limit")
    src = {k: t32(v) for k, v in synth.uniform_box_scene(1, 4).items()}
    dst = R.empty_like_set(src, 4)
    keep = torch.ones(4, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert B.cgsr_compact_gaussians_noalloc(0, keep.data_ptr(), R.arrays_struct(src), R.arrays_struct(dst), [], [],
                                            [], s) == 0
    with pytest.raises(B.CgsrError, match="fixed scratch"):
        B.cgsr_compact_gaussians_noalloc((1 << 26) + 1, keep.data_ptr(), R.arrays_struct(src), R.arrays_struct(dst),
                                         [], [], [], s)
