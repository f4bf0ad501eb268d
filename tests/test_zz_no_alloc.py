"""skim_discrepancy_tail_noalloc, the entry point that allocates nothing (its
scratch is a file-scope device array): through the C ABI its tails equal
those of skim_discrepancy_tail, bit for bit (same kernels, same order), on
two calls in a row, the second with fewer seeds and bins (the scratch keeps
the first call's contents), plus an empty seed list; sizes past its scratch
are refused with nothing written."""
import numpy as np
import pytest

from gpu_util import dev, gpu_greedy

pytestmark = pytest.mark.gpu


def _records():
    from workloads.configs import make_config, make_graph
    cfg = make_config("served-skim")
    g = make_graph(cfg)
    seeds, gains, _, sel, tau, sec = gpu_greedy(g, cfg["ell"], cfg["k"], cfg["seed"], [200],
                                                records=True)
    return tau, sec, gains


def _tails(tau, sec, gains, s, bins, rel):
    import torch
    import paper_1408_6282_amd as sk
    from gpu_util import to_dev_u32, to_dev_u64
    t = to_dev_u64(tau[:s]) if s else None
    c = to_dev_u32(sec[:s]) if s else None
    g = to_dev_u64(gains[:s]) if s else None
    want = torch.full((bins + 1,), -1.0, dtype=torch.float64, device=dev())
    got = torch.full((bins + 1,), -1.0, dtype=torch.float64, device=dev())
    sk.skim_discrepancy_tail(t, c, g, bins, rel, want)
    sk.skim_discrepancy_tail_noalloc(t, c, g, bins, rel, got)
    torch.cuda.synchronize()
    return want.cpu().numpy(), got.cpu().numpy()


def test_noalloc_tail_equals_the_allocating_call_twice():
    tau, sec, gains = _records()
    for s, bins, rel in [(200, 4096, 0.25), (37, 512, 0.1), (0, 64, 0.5)]:
        want, got = _tails(tau, sec, gains, s, bins, rel)
        assert np.array_equal(got, want), (s, bins)
        assert got[0] == 1.0


def test_noalloc_tail_refuses_sizes_past_its_scratch():
    import torch
    import paper_1408_6282_amd as sk
    from gpu_util import to_dev_u32, to_dev_u64
    tau, sec, gains = _records()
    bins = 8192  # 200 * 8193 cells > 2^20
    out = torch.full((bins + 1,), 7.0, dtype=torch.float64, device=dev())
    with pytest.raises(sk.SkimError) as ei:
        sk.skim_discrepancy_tail_noalloc(to_dev_u64(tau), to_dev_u32(sec), to_dev_u64(gains),
                                         bins, 0.25, out)
    assert ei.value.status == sk.SKIM_EUNSUPPORTED
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == 7.0).all()
