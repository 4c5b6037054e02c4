"""Device memory through the caller's allocator (xrl_set_allocator).

With torch's caching allocator installed, the tree, the plan, the stored near
field, the matvec work arrays, GMRES and the loop structures take their device
memory from torch: torch's allocated-byte counter grows by at least the
stored near field while the handles live and falls back when they are
destroyed.  The results are bitwise those of the hipMalloc path (same
kernels, same launch order)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2409_12375_amd import inputs as I  # noqa: E402
from paper_2409_12375_amd import xrl  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_all(V, T, x, e):
    """Tree, plan, near field, matvec, GMRES and an edge-space product; the
    handles are returned open so the caller can see what they hold."""
    tree = xrl.Tree(V, T)
    plan = xrl.Plan(tree, order=8, precision="mixed", max_cols=6)
    plan.assemble()
    y = plan.matvec(x).clone()
    sol, st = plan.gmres(y, alpha=1.0, beta=0.5, restart=20, rtol=1e-6, max_iter=200)
    loops = xrl.Loops(V, T)
    ve = loops.edge_matvec(plan, e, alpha=1j, beta=0.1)
    torch.cuda.synchronize()
    return (tree, plan, loops), (y, sol.clone(), ve)


def test_torch_allocator_holds_the_library_memory_and_changes_no_result():
    say("case: allocator hand-off, bar 2x2x16 mixed, 3 columns")
    V, T = I.bar(2, 2, 16, size=(1.0, 1.0, 4.0))
    N = len(T)
    x = torch.from_numpy(I.densities(N, 3, np.complex64)).cuda()
    loops0 = xrl.Loops(V, T)
    ne = loops0.info()["n_edges"]
    loops0.close()
    e = torch.from_numpy(I.densities(ne, 2)).cuda()
    handles, ref = run_all(V, T, x, e)
    for h in handles:
        h.close()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    try:
        xrl.use_torch_allocator(True)
        handles, got = run_all(V, T, x, e)
        held = torch.cuda.memory_allocated() - base
        info = handles[1].info()
        say("  torch holds %.1f MB for the library's handles (near field %.1f MB)" % (
            held / 2**20, 4 * info["n_near_entries"] / 2**20))
        assert held >= 4 * info["n_near_entries"]
        for a, b in zip(ref, got):
            assert torch.equal(a, b)
        for h in handles:
            h.close()
        del handles
        torch.cuda.synchronize()
        left = torch.cuda.memory_allocated() - base
        say("  after destroy: %d bytes above the start (the results)" % left)
        res_bytes = sum(t.numel() * t.element_size() for t in got)
        assert left <= res_bytes + (1 << 20)  # the results, in 512-byte blocks
    finally:
        xrl.use_torch_allocator(False)
    # hipMalloc again for new handles
    tree = xrl.Tree(V, T)
    tree.close()
