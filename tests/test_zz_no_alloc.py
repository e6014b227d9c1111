"""The allocation-free entry point against agp_propagate.

agp_propagate_noalloc keeps every buffer in the library's fixed per-device
array: its results must equal agp_propagate's bit for bit, on two calls in a
row (the second smaller, so it starts from the first one's leftovers), it
must not change the device's free memory, and it must refuse sizes beyond
the array with AGP_EINVAL.
"""
import gc

import numpy as np
import pytest

from paper_2106_03058_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_03058_amd import agp

    agp.lib()
    g = inputs.chung_lu(20000, 10, 2.3, seed=31, self_loops=True)
    return torch, agp, g, agp.Graph.from_inputs(g, validate=True)


CASES = [
    # (a, b, weights, eps, columns, signal)
    (0.5, 0.5, inputs.weights_hkpr(5.0, 10), 1e-5, 40, "normal"),
    (0.5, 0.5, inputs.weights_hkpr(5.0, 10), 1e-5, 7, "normal"),
    (0.0, 1.0, inputs.weights_ppr(0.2, 12), 1e-6, 16, "onehot"),
    (0.0, 1.0, inputs.weights_ppr(0.2, 12), 1e-6, 3, "onehot"),
]


def _signal(torch, g, C, kind, seed):
    if kind == "onehot":
        src = inputs.sources_uniform(g, C, seed=seed)
        x = np.zeros((g.n, C), dtype=np.float32)
        x[src, np.arange(C)] = 1.0
    else:
        x = inputs.features_normal(g.n, C, seed=seed)
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def test_noalloc_equals_propagate_two_calls_in_a_row(env):
    torch, agp, g, G = env
    for k, (a, b, w, eps, C, kind) in enumerate(CASES):
        X = _signal(torch, g, C, kind, seed=40 + k)
        qids = np.arange(1000 * k, 1000 * k + C, dtype=np.uint32)
        print(f"case {k}: a={a} b={b} C={C} {kind}", flush=True)
        ref, _ = agp.propagate(G, a, b, w, X, eps, 77 + k, qids=qids)  # makes the tables of (a, b)
        out = torch.full_like(X, float("nan"))
        # objects of earlier tests that the collector frees (graphs, servers)
        # return their memory: collect them first and keep the collector off
        # while the call is measured
        gc.collect()
        torch.cuda.synchronize()
        gc.disable()
        try:
            free0 = torch.cuda.mem_get_info()[0]
            agp.propagate_noalloc(G, a, b, w, X, eps, 77 + k, qids=qids, out=out)
            torch.cuda.synchronize()
            free1 = torch.cuda.mem_get_info()[0]
        finally:
            gc.enable()
        assert free1 == free0, "the call changed the device's free memory"
        assert torch.equal(out, ref), f"case {k}: max diff {(out - ref).abs().max().item()}"


def test_noalloc_rejects_what_does_not_fit(env):
    torch, agp, g, G = env
    C = agp.NOALLOC_SCRATCH_BYTES // (32 * g.n) + 1  # 32 bytes per cell
    X = torch.zeros((g.n, C), dtype=torch.float32, device="cuda:0")
    X[0] = 1.0
    with pytest.raises(agp.AGPError) as e:
        agp.propagate_noalloc(G, 0.0, 1.0, inputs.weights_ppr(0.2, 5), X, 1e-4, 1)
    assert e.value.code == agp.AGP_EINVAL and "cells" in str(e.value)
    # and a call that fits still works afterwards
    X2 = _signal(torch, g, 5, "normal", seed=3)
    ref, _ = agp.propagate(G, 0.5, 0.5, inputs.weights_hkpr(5.0, 10), X2, 1e-5, 9)
    got = agp.propagate_noalloc(G, 0.5, 0.5, inputs.weights_hkpr(5.0, 10), X2, 1e-5, 9)
    assert torch.equal(got, ref)


def test_noalloc_needs_the_tables(env):
    torch, agp, g, G = env
    X = _signal(torch, g, 2, "normal", seed=5)
    with pytest.raises(agp.AGPError) as e:  # exponents no earlier call used
        agp.propagate_noalloc(G, 0.37, 0.63, inputs.weights_ppr(0.2, 4), X, 1e-4, 1)
    assert e.value.code == agp.AGP_EINVAL
