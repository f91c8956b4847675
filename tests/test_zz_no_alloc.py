"""The allocation-free entry point (qk_overlap_gram_noalloc) against
qk_overlap_gram on the same batches: the same kernels run, with the
refinement masks (tile sweeps) and pair lists (large-bond sweep) in the
library's static device scratch instead of stream-ordered allocations, so
every output must be bitwise equal. Two calls in a row per form, the second
on a smaller input (the scratch keeps the first call's contents), and a call
that needs more scratch than the array holds is rejected before anything is
enqueued. The first call's outputs are also held to the oracle's gates."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import checks, mps  # noqa: E402
from synthdata import gen_clusters  # noqa: E402
from tests._util import oracle_import_layout  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qk():
    import paper_2602_01330_amd.qk as qk
    return qk


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def both(qk, b, c, symmetric, prec, fuse_x=None):
    """(reference call, allocation-free call) outputs: kq, ln, kc, k."""
    out = []
    for fn in (qk.qk_overlap_gram, qk.qk_overlap_gram_noalloc):
        info_r, info_c = qk.qk_mps_info(b), qk.qk_mps_info(c)
        m, n = info_r["n_samples"], info_c["n_samples"]
        f64 = dict(dtype=torch.float64, device="cuda")
        kq = torch.full((m, n), float("nan"), **f64)
        ln = torch.full((m, n), float("nan"), **f64)
        fuse = None
        if fuse_x is not None:
            xr, xc = fuse_x
            fuse = {"x_rows": xr, "x_cols": xc, "gamma": 1.0 / xr.shape[1], "w": 0.25,
                    "kc": torch.full((m, n), float("nan"), **f64),
                    "k": torch.full((m, n), float("nan"), **f64)}
        fn(b, c, symmetric, prec, kq, ln, fuse)
        torch.cuda.synchronize()
        res = [kq.cpu().numpy(), ln.cpu().numpy()]
        if fuse is not None:
            res += [fuse["kc"].cpu().numpy(), fuse["k"].cpu().numpy()]
        out.append(res)
    return out


@pytest.mark.parametrize("prec", ["fp32_mfma", "fp32", "bf16x3", "fp64", "auto"])
def test_small_bond_forms_two_calls(qk, prec):
    """Bond 4 (d = 64, L = 2): tile sweeps with the FP64 refinement of pairs
    above tau (masks in the scratch); 77 then 37 rows (ragged tiles)."""
    X, _ = gen_clusters(77, 64, 4242)
    Y, _ = gen_clusters(50, 64, 4343)
    for n_rows, sym in ((77, True), (37, False)):
        xr = dev(X[:n_rows])
        xc = xr if sym else dev(Y)
        b = qk.qk_mps_build(xr, 2, 64)
        c = b if sym else qk.qk_mps_build(xc, 2, 64)
        print(f"[noalloc] {prec} rows={n_rows} symmetric={sym}", flush=True)
        ref, got = both(qk, b, c, sym, prec, (xr, xc))
        for a, g in zip(ref, got):
            assert np.array_equal(a, g, equal_nan=False), prec
        if n_rows == 77:
            P = mps.pad_batch(mps.build_batch(X[:n_rows], 2, 64))
            K, LN = mps.gram(P, P, symmetric=True)
            assert checks.gate_a(got[0], K)[0] and checks.gate_b(got[1], LN)[0]
        for x in {id(b): b, id(c): c}.values():
            x.close()


def test_large_bond_matrix_core_two_calls(qk):
    """Bond 16 (oracle-built MPS, d = 10, L = 4): the matrix-core sweep with
    its FP64 list pass (pair list in the scratch); 9 x 9 symmetric, then a
    smaller 5 x 9 rectangle."""
    X, _ = gen_clusters(9, 10, 310)
    Y, _ = gen_clusters(5, 10, 410)
    MX, MY = mps.build_batch(X, 4, 64), mps.build_batch(Y, 4, 64)
    cx, tx = oracle_import_layout(MX, 16)
    cy, ty = oracle_import_layout(MY, 16)
    bx = qk.qk_mps_import(cx, tx, 4, 64)
    by = qk.qk_mps_import(cy, ty, 4, 64)
    for b, c, sym in ((bx, bx, True), (by, bx, False)):
        print(f"[noalloc] wide symmetric={sym}", flush=True)
        ref, got = both(qk, b, c, sym, "fp32_mfma")
        for a, g in zip(ref, got):
            assert np.array_equal(a, g)
        _, LN = mps.gram(mps.pad_batch(MX if sym else MY), mps.pad_batch(MX), symmetric=sym)
        assert checks.gate_b(got[1], LN)[0]
        if sym:
            assert np.abs(np.diag(got[0]) - 1.0).max() <= 1e-5
    bx.close()
    by.close()


def test_oversized_call_is_rejected_before_launch(qk):
    """15,440 samples symmetric at bond 2: 965 tile rows, 466,095 tiles, whose
    masks need 16,779,424 bytes, more than the 16 MiB scratch: INVALID_ARG,
    and the outputs stay untouched."""
    n = 15440
    rng = np.random.default_rng(9)
    x = dev(rng.uniform(0.0, np.pi, size=(n, 2)))
    b = qk.qk_mps_build(x, 1, 16)
    ln = torch.full((n, n), float("nan"), dtype=torch.float64, device="cuda")
    with pytest.raises(qk.QkError, match="scratch"):
        qk.qk_overlap_gram_noalloc(b, b, True, "fp32_mfma", None, ln)
    torch.cuda.synchronize()
    assert bool(torch.isnan(ln[:4, :4]).all()) and bool(torch.isnan(ln[-4:, -4:]).all())
    b.close()
