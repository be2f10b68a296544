"""GPU tests of shared-table plans (cip_plan_attach) and of the request
server (cip_server_*): every result is the same alone and in the mix
(bit for bit: the same kernels run on the same data), one result is checked
against the FP64 oracle, and admission respects the HBM budget."""
import threading

import numpy as np
import pytest
import torch

from tests import parity
from oracle import admm, model
from paper_2006_08303_amd import cip, synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
MiB = 1 << 20


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=DEV)


def _meas(N, K, S, cfg, idx):
    """Measurements of a smooth scene through disk kernels at 30 dB."""
    x, psf, _ = synth.problem("smooth_disk", N, K, S, seed_config=cfg)
    noise = synth.unit_noise(synth.rng_for(cfg, 100 + idx), K, N, N)
    hx = model.forward(x, psf)
    y = hx + model.snr_noise_scale(hx, 30.0)[:, None, None] * noise
    return psf, y.astype(np.float32)


def test_attached_plans_run_concurrently():
    N, K, S = 256, 3, 3
    psf, y0 = _meas(N, K, S, 5, 0)
    _, y1 = _meas(N, K, S, 5, 1)
    base = cip.Plan(_t(psf), "tv3d", 1e-2, 1e-3, 1.0)
    ref0 = base.solve(_t(y0), 20).clone()
    ref1 = base.solve(_t(y1), 20).clone()
    a, b = base.attach(), base.attach()
    s0, s1 = torch.cuda.Stream(), torch.cuda.Stream()
    ya, yb = _t(y0), _t(y1)
    torch.cuda.synchronize()
    xa = a.solve(ya, 20, stream=s0)
    xb = b.solve(yb, 20, stream=s1)
    torch.cuda.synchronize()
    assert torch.equal(xa, ref0) and torch.equal(xb, ref1)


SPEC = [("tv3d", 256, 3, 3), ("tv3d", 128, 5, 5), ("dct2d", 512, 3, 3), ("tv3d", 64, 8, 8),
        ("wdct3d", 128, 3, 3)]


def _server_with_ops(budget, slots):
    srv = cip.Server(budget, n_slots=slots)
    ops, psfs = [], []
    for j, (prior, N, K, S) in enumerate(SPEC):
        psf, _ = _meas(N, K, S, 5, 0)
        rho, lam = (1e-2, 1e-3) if prior == "tv3d" else (0.1, 1e-2)
        ops.append(srv.add_operator(_t(psf), prior, rho, lam, 1.0))
        psfs.append(psf)
    return srv, ops, psfs


def _requests():
    reqs = []
    for i in range(12):
        j = i % len(SPEC)
        prior, N, K, S = SPEC[j]
        _, y = _meas(N, K, S, 5, 10 + i)
        reqs.append((j, y, 5 + 3 * (i % 4)))
    return reqs


def test_server_mix_equals_alone():
    reqs = _requests()
    # alone: one slot, one request at a time
    srv, ops, _ = _server_with_ops(4096 * MiB, 1)
    alone = []
    for j, y, it in reqs:
        prior, N, K, S = SPEC[j]
        x = np.full((S, N, N), np.nan, np.float32)
        srv.wait(srv.submit(ops[j], y, x, it))
        alone.append(x)
    srv.close()
    # mix: four slots, everything submitted at once from two threads
    srv, ops, _ = _server_with_ops(4096 * MiB, 4)
    outs = [np.full((SPEC[j][3], SPEC[j][1], SPEC[j][1]), np.nan, np.float32) for j, _, _ in reqs]
    tickets = [None] * len(reqs)

    def submit(idx):
        for i in idx:
            j, y, it = reqs[i]
            tickets[i] = srv.submit(ops[j], y, outs[i], it)

    th = [threading.Thread(target=submit, args=(range(k, len(reqs), 2),)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    lat = [srv.wait(t)[0] for t in tickets]
    srv.close()
    print(f"mix latencies: max {max(lat) * 1e3:.1f} ms", flush=True)
    for i, (a, b) in enumerate(zip(alone, outs)):
        assert np.array_equal(a, b), i


def test_server_result_matches_oracle():
    prior, N, K, S = SPEC[1]
    psf, y = _meas(N, K, S, 5, 0)
    srv = cip.Server(1024 * MiB, n_slots=2)
    op = srv.add_operator(_t(psf), prior, 1e-2, 1e-3, 1.0)
    x = np.zeros((S, N, N), np.float32)
    srv.wait(srv.submit(op, y, x, 10))
    srv.close()
    ref = admm.AnalysisADMM(psf.astype(np.float64), "tv3d", 1e-3, 1e-2, 1.0,
                            tier="freq").run(y.astype(np.float64), 10)[0]
    err = admm.rel_l2(x.astype(np.float64), ref)
    print(f"  rel_l2 = {err:.3e}", flush=True)
    parity.check(x.astype(np.float64), ref, 1e-4)


def test_server_admission_by_footprint():
    """A budget that holds the operator and one request at a time: all
    requests still finish (queued until memory frees up) with the lone-solve
    result; an operator or a request that can never fit is refused."""
    prior, N, K, S = "tv3d", 256, 3, 3
    psf, y = _meas(N, K, S, 5, 0)
    def r256(b):
        return (b + 255) // 256 * 256

    ws = cip.workspace_bytes(K, S, N, N, prior)
    base = cip.Plan(_t(psf), prior, 1e-2, 1e-3, 1.0)
    ref = base.solve(_t(y), 8).cpu().numpy()
    st = base.attach().workspace.numel()      # solve-state bytes of this operator
    req = r256(st) + r256(K * N * N * 4) + r256(S * N * N * 4)
    srv = cip.Server(r256(ws) + req + req // 2, n_slots=4)
    op = srv.add_operator(_t(psf), prior, 1e-2, 1e-3, 1.0)
    outs = [np.zeros((S, N, N), np.float32) for _ in range(6)]
    ts = [srv.submit(op, y, o, 8) for o in outs]
    waits = [srv.wait(t) for t in ts]
    for o in outs:
        assert np.array_equal(o, ref)
    assert max(q for _, q in waits) > 0.0
    psf2, _ = _meas(512, K, S, 5, 0)
    with pytest.raises(cip.CipError) as e:        # a larger operator does not fit
        srv.add_operator(_t(psf2), prior, 1e-2, 1e-3, 1.0)
    assert e.value.code == -3
    srv.close()
    small = cip.Server(ws + 64 * 1024, n_slots=1)   # operator fits, no request can
    op = small.add_operator(_t(psf), prior, 1e-2, 1e-3, 1.0)
    with pytest.raises(cip.CipError) as e:
        small.submit(op, y, outs[0], 8)
    assert e.value.code == -3
    small.close()
