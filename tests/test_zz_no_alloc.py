"""GPU check of jevd_adjoint_noalloc (the adjoint on the library's fixed
scratch array, for callers that cannot allocate) through the C ABI: two
calls in a row, the second on a smaller input, each against jevd_adjoint on
the same inputs (same kernels and arithmetic, so bit for bit); sizes beyond
the fixed scratch are refused before any device work.  Needs an MI355X."""
import numpy as np
import pytest

from paper_1008_0201_amd import workloads as W

pytestmark = pytest.mark.gpu
SCRATCH_DOUBLES = 4 << 20


def _inputs(torch, count, m, n, k):
    from paper_1008_0201_amd.autograd import eigh_jacobi
    G, J, w, C = W.adjoint_batch(count=count, n=n, k=k, m=m)
    Gt = torch.from_numpy(G).cuda()
    lam, U = eigh_jacobi(Gt, torch.from_numpy(J).cuda())
    return dict(G=Gt.transpose(1, 2).contiguous(), U=U.transpose(1, 2).contiguous(),
                lam=lam.contiguous(), J=torch.from_numpy(J).cuda(),
                w=torch.from_numpy(w).cuda(),
                C=torch.from_numpy(np.ascontiguousarray(C.transpose(0, 2, 1))).cuda())


def _call(B, fn, h, x, count, m, n, out):
    return fn(h, count, m, n, x["G"].data_ptr(), m, m * n, x["J"].data_ptr(), n,
              x["lam"].data_ptr(), n, x["U"].data_ptr(), m, m * n, x["w"].data_ptr(), n,
              x["C"].data_ptr(), m, m * n, out.data_ptr(), m, m * n)


def test_noalloc_adjoint_matches_the_allocating_entry_point():
    import torch
    from paper_1008_0201_amd import jevd as B
    assert torch.cuda.is_available()
    s = B.Solver()
    try:
        for count, m, n, k in [(12, 150, 128, 31), (3, 70, 50, 32)]:   # second call smaller
            x = _inputs(torch, count, m, n, k)
            ref = torch.full((count, n, m), 7.0, dtype=torch.float64, device="cuda")
            got = torch.full((count, n, m), -7.0, dtype=torch.float64, device="cuda")
            assert _call(B, B.jevd_adjoint_noalloc, s.h, x, count, m, n, got) == B.JEVD_OK
            assert _call(B, B.jevd_adjoint, s.h, x, count, m, n, ref) == B.JEVD_OK
            torch.cuda.synchronize()
            g, r = got.cpu().numpy(), ref.cpu().numpy()
            assert np.all(np.isfinite(r))
            assert np.array_equal(g, r), (count, m, n, float(np.max(np.abs(g - r))))
    finally:
        s.close()


def test_noalloc_adjoint_refuses_sizes_beyond_its_scratch():
    import torch
    from paper_1008_0201_amd import jevd as B
    s = B.Solver()
    try:
        n = m = 512
        per = 3 * n * n + m * n                       # 1 MiB doubles per instance
        count = SCRATCH_DOUBLES // per + 1            # one instance too many
        st = B.jevd_adjoint_noalloc(s.h, count, m, n, 8, m, m * n, 0, n, 8, n, 8, m, m * n, 0, n,
                                    0, m, m * n, 8, m, m * n)
        assert st == B.JEVD_EINVAL                    # refused on the host: no device work
        torch.cuda.synchronize()
    finally:
        s.close()
