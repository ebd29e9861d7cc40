"""rrt_relight_noalloc (relight with the library's own scratch array instead
of a caller workspace) against rrt_relight with a caller workspace, through
the C ABI: bit-identical radiance on two calls in a row, the second with a
smaller input (the scratch keeps the first call's contents), and both
within the FP32 bar of the FP64 checker."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rrt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_07272_amd as m
    return m


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def _inputs(case):
    return (_dev(case["light_idx"]), _dev(case["light_val"]), _dev(case["vert_rot"]),
            _dev(case["t_idx"]), _dev(case["t_val"]),
            None if case["frame_rot"] is None else _dev(case["frame_rot"]))


# (workload seed, n, top-k lighting, vertices, transport nnz, frames, flags):
# the second case is smaller than the first in every size
CASES = [(31, 128, 1024, 300, 256, 2, dict(compensated=False)),
         (32, 32, 256, 40, 64, 1, dict(compensated=True))]


def test_noalloc_matches_relight_twice(rrt):
    from cases import build_case, frame_errors, reference, workload
    for seed, n, k, nv, nnz, nf, flags in CASES:
        print(f"noalloc case n={n} V={nv} F={nf} nnz={nnz} {flags}", flush=True)
        case = build_case(workload(seed, n, k, nv, nnz, nframes=nf))
        li, lv, rot, ti, tv, frot = _inputs(case)
        want = rrt.relight(n, li, lv, rot, ti, tv, frame_rot=frot, **flags)
        got = torch.full_like(want, float("nan"))
        rrt.relight_noalloc(n, li, lv, rot, ti, tv, out=got, frame_rot=frot, **flags)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (got - want).abs().max().item()
        errs = frame_errors(got.cpu().numpy(), reference(case))
        assert max(errs) <= 1e-5, errs


def test_noalloc_chain_rule_after_plain(rrt):
    """The chain rule keeps its block coefficients in the staging part of the
    scratch: a chain-rule call after a plain one still equals rrt_relight."""
    from cases import build_case, workload
    case = build_case(workload(33, 64, 512, 64, 128))
    li, lv, rot, ti, tv, _ = _inputs(case)
    out = torch.empty((1, rot.shape[0]), dtype=torch.float32, device="cuda")
    for chain in (False, True, False):
        print(f"noalloc n=64 chain_rule={chain}", flush=True)
        want = rrt.relight(64, li, lv, rot, ti, tv, chain_rule=chain)
        rrt.relight_noalloc(64, li, lv, rot, ti, tv, out=out, chain_rule=chain)
        torch.cuda.synchronize()
        assert torch.equal(out, want)
