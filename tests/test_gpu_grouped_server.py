"""GPU parity of the grouped persistent GEMM and of the serving runtime."""
import numpy as np
import pytest

import oracle as orc
from paper_2602_10262_amd import synth
from tests.helpers import check_gemm, check_gemm_sampled, dev, host, log

pytestmark = pytest.mark.gpu


def _mix(seed, specs):
    """Problems (M, N, K, sparse) with quantized operands built by the oracle."""
    probs = []
    for i, (M, N, K, sparse) in enumerate(specs):
        xa = synth.normal_outliers(seed * 100 + 2 * i, (M, K))
        xw = synth.normal_outliers(seed * 100 + 2 * i + 1, (N, K))
        qa, _, da = orc.quantize(xa, 0, True)
        qw, _, dw = orc.quantize(xw, 0, True)
        if sparse:
            v, m, _, qw = orc.prune24(qw, 0)
        else:
            v = m = None
        probs.append(dict(M=M, N=N, K=K, sparse=sparse, qa=qa, da=da, qw=qw, dw=dw, v=v, m=m))
    return probs


def _gproblems(gpu, probs):
    import torch
    out = []
    for p in probs:
        a, da, dw = dev(p["qa"]), dev(p["da"]), dev(p["dw"])
        c = torch.full((p["M"], p["N"]), float("nan"), dtype=torch.bfloat16, device="cuda")
        if p["sparse"]:
            v, m = dev(p["v"]), dev(p["m"])
            gp = gpu.sparse_weight_problem(a, v, m, da, dw, c)
            keep = (a, v, m, da, dw)
        else:
            w = dev(p["qw"])
            gp = gpu.dense_problem(a, w, da, dw, c)
            keep = (a, w, da, dw)
        p["c"] = c
        p["keep"] = keep
        out.append(gp)
    return out


# small K: these run on the exact-sum list whatever the plan's tile
SPECS = [(1, 256, 512, False), (37, 384, 256, True), (200, 256, 1024, False), (5, 512, 512, True),
         (300, 128, 384, True), (64, 640, 256, False), (17, 256, 768, False), (129, 256, 512, True)]
# K >= 3584: these run on the plan's FP8 tile
SPECS_LONG_K = [(1, 256, 4096, False), (37, 384, 3584, True), (200, 256, 4096, False), (5, 512, 4096, True),
                (300, 128, 3712, True), (64, 640, 3600, False)]


@pytest.mark.parametrize("tile", [0, 7, 9, 12, 13, 17, 19, 23, 26])
def test_grouped_matches_oracle(gpu, tile):
    import torch
    probs = _mix(1, SPECS + SPECS_LONG_K)
    plan = gpu.GroupedPlan(_gproblems(gpu, probs), tile=tile)
    log(f"grouped tile={tile} info={plan.info()}")
    plan.run()
    torch.cuda.synchronize()
    for p in probs:
        check_gemm(p["c"], p["qa"], 0, p["qw"], 0, p["da"], p["dw"], True,
                   f"grouped M={p['M']} N={p['N']} K={p['K']} sparse={p['sparse']}")
    plan.close()


def test_grouped_graph_replays_equal_eager_and_alone(gpu):
    import torch
    probs = _mix(2, SPECS)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        eager = gpu.GroupedPlan(_gproblems(gpu, probs), tile=12)
        eager.run(st)
        st.synchronize()
        ref = [p["c"].clone() for p in probs]
        graph = gpu.GroupedPlan(_gproblems(gpu, probs), tile=12, use_graph=True)
        for rep in range(4):
            for p in probs:
                p["c"].fill_(float("nan"))       # eager work between replays
            st.synchronize()
            graph.run(st)
            st.synchronize()
            for p, r in zip(probs, ref):
                assert torch.equal(p["c"], r), f"replay {rep}"
        # each problem alone in a one-problem launch gives the same bits
        for i, p in enumerate(probs):
            alone = _mix(2, SPECS)[i]
            one = gpu.GroupedPlan(_gproblems(gpu, [alone]), tile=12)
            one.run(st)
            st.synchronize()
            assert torch.equal(alone["c"], ref[i]), i
            one.close()
        graph.close()
        eager.close()


def test_server_results_same_alone_and_in_mix(gpu):
    """Requests of mixed sizes on 4 streams; every result equals the oracle
    (bound) and equals the same request run alone, bit for bit."""
    import torch
    rng = np.random.default_rng(5)
    Ws = []
    for i, (N, K, sparse) in enumerate([(512, 256, False), (256, 512, True), (384, 384, False)]):
        xw = synth.normal_outliers(500 + i, (N, K))
        qw, _, dw = orc.quantize(xw, 0, True)
        v = m = None
        if sparse:
            v, m, _, qw = orc.prune24(qw, 0)
        Ws.append(dict(N=N, K=K, sparse=sparse, qw=qw, dw=dw, v=v, m=m))
    reqs = []
    for r in range(40):
        wi = int(rng.integers(0, 3))
        M = int(synth.log_uniform_int(rng, 1, 300, 1)[0])
        x = synth.normal_outliers(900 + r, (M, Ws[wi]["K"]))
        reqs.append(dict(w=wi, M=M, x=x))

    def run(num_streams, max_inflight, subset):
        srv = gpu.Server(1 << 28, num_streams, max_inflight)
        dev_w = []
        for W in Ws:
            if W["sparse"]:
                t = (dev(W["v"]), dev(W["m"]), dev(W["dw"]))
                wid = srv.register_weight(t[0], t[1], t[2], W["N"], W["K"])
            else:
                t = (dev(W["qw"]), None, dev(W["dw"]))
                wid = srv.register_weight(t[0], None, t[2], W["N"], W["K"])
            dev_w.append((wid, t))
        outs, keep, tickets = {}, [], []
        for i in subset:
            R = reqs[i]
            xd = dev(R["x"])
            c = torch.full((R["M"], Ws[R["w"]]["N"]), float("nan"), dtype=torch.bfloat16, device="cuda")
            keep.append(xd)
            outs[i] = c
            # the server's streams are not ordered after torch's: x and c
            # must be complete before the request is submitted
            torch.cuda.current_stream().synchronize()
            tickets.append(srv.submit(R["M"], dev_w[R["w"]][0], xd, c))
        for t in tickets:
            assert srv.wait(t, 30_000_000) == gpu.FP8_OK
        st = srv.stats()
        srv.close()
        return outs, st

    mix, st = run(4, 0, range(len(reqs)))
    log(f"server mix stats: {st}")
    assert st["done"] == len(reqs)
    for i in range(0, len(reqs), 3):
        alone, _ = run(1, 1, [i])
        assert torch.equal(alone[i], mix[i]), i
    for i in range(0, len(reqs), 4):
        R, W = reqs[i], Ws[reqs[i]["w"]]
        qa, _, da = orc.quantize(R["x"], 0, True)
        check_gemm(mix[i], qa, 0, W["qw"], 0, da, W["dw"], True, f"request {i} M={R['M']}")


def test_grouped_config4_shapes_match_standalone_and_oracle(gpu):
    """Transformer-shaped problems of the grouped workload (tokens up to 4096,
    (N, K) from the four weight shapes, half of them 2:4 on the weight side)
    in one grouped plan with the library's default tile: every problem's
    result equals the same problem run by fp8_gemm / fp8_sparse24_gemm with
    that tile and no split, bit for bit, and sampled outputs meet the bound
    against the oracle."""
    import torch
    specs = [(4096, 14336, 4096, False), (300, 4096, 14336, True), (1, 4096, 4096, False), (17, 12288, 4096, True),
             (1000, 4096, 14336, False), (64, 14336, 4096, True), (2048, 12288, 4096, False), (5, 4096, 4096, True)]
    probs = []
    for i, (M, N, K, sparse) in enumerate(specs):
        xa = synth.normal_outliers(7000 + 2 * i, (M, K))
        xw = synth.normal_outliers(7001 + 2 * i, (N, K))
        qa, _, da = orc.quantize(xa, 0, True)
        qw, _, dw = orc.quantize(xw, 0, True)
        del xa, xw
        v = m = None
        if sparse:
            v, m, _, qw = orc.prune24(qw, 0)
        probs.append(dict(M=M, N=N, K=K, sparse=sparse, qa=qa, da=da, qw=qw, dw=dw, v=v, m=m))
    plan = gpu.GroupedPlan(_gproblems(gpu, probs))
    info = plan.info()
    log(f"grouped config-4 subset: {info}")
    plan.run()
    torch.cuda.synchronize()
    tile = info["tile"]
    for p in probs:
        a, da, dw = p["keep"][0], p["keep"][-2], p["keep"][-1]
        if p["sparse"]:
            alone = gpu.fp8_sparse24_gemm(p["keep"][1], p["keep"][2], a, gpu.FP8_SPARSE_B, da, dw,
                                          out_dtype=torch.bfloat16, plan=(tile, 1))
        else:
            alone = gpu.fp8_gemm(a, p["keep"][1], da, dw, out_dtype=torch.bfloat16, plan=(tile, 1))
        torch.cuda.synchronize()
        what = f"M={p['M']} N={p['N']} K={p['K']} sparse={p['sparse']}"
        assert torch.equal(alone.view(torch.int16), p["c"].view(torch.int16)), what
        check_gemm_sampled(p["c"], p["qa"], 0, p["qw"], 0, p["da"], p["dw"], True, n=512, what="grouped " + what)
    plan.close()
