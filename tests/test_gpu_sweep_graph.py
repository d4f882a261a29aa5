"""Monte-Carlo sweep points replayed from HIP graphs (the chunk pipeline of
the Eb/N0 sweeps, Sec. 6.1: random bits, direct encoding, BPSK/AWGN, int8
quantisation, decoding, fallback re-decoding, error counting) give exactly
the counters of the same stages called eagerly; the device-resident seed
that makes the replays possible reproduces the host-seeded generators."""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2306_12063_amd as P
from paper_2306_12063_amd import learned

pytestmark = pytest.mark.gpu
DEV = "cuda"


def test_device_seed_equals_host_seed():
    h = synth.wifi_code("1/2", 27)
    F, K, N = 37, 324, 648
    for seed in (0, 5, (1 << 63) + 12345):
        sd = torch.tensor([seed - (1 << 64) if seed >= 1 << 63 else seed], dtype=torch.int64, device=DEV)
        a = P.ldpc_random_bits(seed, F, K)
        b = P.ldpc_random_bits(sd, F, K)
        assert torch.equal(a, b)
        cw = P.ldpc_encode(h, 27, a)
        la = P.ldpc_awgn_llr(seed, cw, 0.8, 3.125)
        lb = P.ldpc_awgn_llr(sd, cw, 0.8, 3.125)
        assert torch.equal(la, lb)
    # and against the oracle's Philox stream
    got = P.ldpc_random_bits(torch.tensor([9], dtype=torch.int64, device=DEV), F, K).cpu().numpy()
    assert np.array_equal(got, oracle.frame_bits(9, F, K))


@pytest.mark.parametrize("kind,rate,Z", [("wifi", "1/2", 27), ("wimax", "2/3A", 48)])
def test_graph_sweep_equals_eager(kind, rate, Z):
    h = synth.wifi_code(rate, Z) if kind == "wifi" else synth.wimax_code(rate, Z)
    Mb, Nb = h.shape
    rng = np.random.default_rng(3)
    w = torch.from_numpy(rng.uniform(0.55, 0.95, (10, Mb, Nb)).astype(np.float32)).to(DEV)
    decs = learned.decoders(h, Z, w)
    pts = [1.0, 2.0, 3.0]
    g = learned.sweep(h, Z, decs, pts, 2048, chunk=1024, seed=11, graph=True)
    e = learned.sweep(h, Z, decs, pts, 2048, chunk=1024, seed=11, graph=False)
    for name in g:
        for pg, pe in zip(g[name], e[name]):
            assert pg["counters_first"] == pe["counters_first"], (name, pg["ebn0"])
            assert pg["counters_final"] == pe["counters_final"], (name, pg["ebn0"])
            assert pg["gbit_s"] > 0
    # the sweep measured something: errors fall with Eb/N0 for plain NMS
    fer = [p["fer"] for p in g["plain_nms_f32"]]
    assert fer[0] >= fer[-1]


def test_graph_replays_repeat():
    """The captured stages replayed twice for one point, with eager work and
    synchronisations between, reproduce the counters and the decoded bits."""
    h = synth.wifi_code("5/6", 27)
    w = torch.full((10, 4, 24), 0.75, dtype=torch.float32, device=DEV)
    decs = learned.decoders(h, 27, w)
    pipe = learned.SweepPipeline(h, 27, decs, 512)
    pipe.set_point(3.0, 99)
    pipe.capture()
    results = []
    for rep in range(3):
        pipe.clear_counters()
        pipe.set_point(3.0, 99)
        ev = []
        pipe.run_chunk(ev)
        torch.cuda.synchronize()
        _ = torch.ones(1000, device=DEV).sum().item()   # eager work between replays
        results.append({n: (o["first"].clone(), o["final"].clone(), o["bits"].clone()) for n, o in pipe.out.items()})
    for r in results[1:]:
        for n in r:
            for a, b in zip(r[n], results[0][n]):
                assert torch.equal(a, b), n
    # the eager stages on the same buffers give the same counters
    pipe.graphs = None
    pipe.clear_counters()
    pipe.set_point(3.0, 99)
    pipe.run_chunk([])
    torch.cuda.synchronize()
    for n, o in pipe.out.items():
        assert torch.equal(o["first"], results[0][n][0]) and torch.equal(o["final"], results[0][n][1]), n
