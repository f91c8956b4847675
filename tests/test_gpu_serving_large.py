"""Serving at the large feature dimensions of the served workload (d = 256
and 784 qubits, cluster inputs, L = 2, chi_max 64): K_q there lies far below
1e-8 off the diagonal and partly below the FP64 range, so the rows are
compared in the log domain, through the ln K_q rows a request can ask for
(QK_OUT_LNKQ), under the stated log gate against the FP64 oracle; w = 1
requests return K_q itself. Also: a request whose encoding latches a device
check (the SVD sweep limit) fails with the check's text instead of
returning rows."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import checks, classical, mps  # noqa: E402
from synthdata import config_inputs  # noqa: E402

pytestmark = pytest.mark.gpu

NSUP = 40


@pytest.fixture(scope="module")
def qk():
    import paper_2602_01330_amd.qk as qk
    return qk


def oracle_ln_rows(x, sup):
    A = mps.pad_batch(mps.build_batch(x, 2, 64))
    B = mps.pad_batch(mps.build_batch(sup, 2, 64))
    return mps.gram(A, B)


@pytest.mark.parametrize("d", [256, 784])
def test_large_d_rows_in_the_log_domain(qk, d):
    sup, test, _ = config_inputs("C5", d=d, n_train=NSUP, n_test=8)
    srv = qk.qk_server_create()
    try:
        qk.qk_server_load_support(srv, torch.as_tensor(sup, device="cuda"), 2, 64)
        plan = [(test[0:3], 1.0), (test[3:4], 1.0), (test[4:8], 0.4)]
        ids = [qk.qk_server_submit_ex(srv, x, w, qk.QK_OUT_LNKQ) for x, w in plan]
        print(f"[serve large] d={d} supports={NSUP} requests={len(plan)}", flush=True)
        for rid, (x, w) in zip(ids, plan):
            assert qk.qk_server_wait(srv, rid, 120000) == qk.QK_REQ_DONE, qk.qk_last_error()
            rows = np.empty((len(x), NSUP))
            ln = np.empty((len(x), NSUP))
            assert qk.qk_server_poll_ex(srv, rid, rows=rows, ln=ln) == qk.QK_REQ_DONE
            K, LN = oracle_ln_rows(x, sup)
            ok_b, lmax = checks.gate_b(ln, LN)
            print(f"[serve large] d={d} rows={len(x)} w={w} max|d lnK|={lmax:.3e} "
                  f"median log10 K_q={np.median(LN) / np.log(10):.1f}", flush=True)
            assert ok_b, lmax
            ref = classical.mix(K, classical.rbf_gram(x, sup, 1.0 / d), w)
            ok_a, dmax, rel = checks.gate_a(rows, ref)
            assert ok_a, (dmax, rel)
            if w == 1.0:  # the rows are K_q = exp(ln K_q) (the device's exp)
                assert np.allclose(rows, np.exp(ln), rtol=1e-13, atol=0.0)
        with pytest.raises(qk.QkError):  # ln rows of a request that did not ask
            rid = qk.qk_server_submit(srv, test[:1], 0.5)
            assert qk.qk_server_wait(srv, rid, 120000) == qk.QK_REQ_DONE
            qk.qk_server_poll_ex(srv, rid, ln=np.empty((1, NSUP)))
    finally:
        srv.close()


def test_latched_build_check_fails_the_request(qk):
    """With the SVD sweep limit at 0, every two-site SVD that needs a rotation
    reports non-convergence, so the request's build latches the flag: the
    request ends FAILED with the flag's text. Back at the default limit the
    same rows are served and match the oracle."""
    d = 16
    sup, test, _ = config_inputs("C5", d=d, n_train=24, n_test=4)
    srv = qk.qk_server_create()
    try:
        qk.qk_server_load_support(srv, torch.as_tensor(sup, device="cuda"), 2, 64)
        qk.qk_set_svd_sweep_limit(0)
        try:
            rid = qk.qk_server_submit(srv, test, 0.5)
            st = qk.qk_server_wait(srv, rid, 60000)
            assert st == qk.QK_REQ_FAILED
            st2, rows = qk.qk_server_poll(srv, rid, np.empty((4, 24)))
            assert st2 == qk.QK_REQ_FAILED and rows is None
            assert "sweep limit" in qk.qk_last_error()
        finally:
            qk.qk_set_svd_sweep_limit(60)
        rid = qk.qk_server_submit(srv, test, 0.5)
        assert qk.qk_server_wait(srv, rid, 60000) == qk.QK_REQ_DONE
        out = np.empty((4, 24))
        st, rows = qk.qk_server_poll(srv, rid, out)
        K, _ = oracle_ln_rows(test, sup)
        ok, dmax, rel = checks.gate_a(rows, classical.mix(K, classical.rbf_gram(test, sup, 1 / d), 0.5))
        assert ok, (dmax, rel)
    finally:
        srv.close()
