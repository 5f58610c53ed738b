"""Helpers for the GPU parity tests (host-side marshalling only)."""
import numpy as np
import torch

import oracle
import paper_1105_4490_amd as P


def dev_h(h):
    return P.DeviceHypergraph.from_host(h)


def dev_x(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32)).cuda().contiguous()


def host(t):
    return None if t is None else t.cpu().numpy()


def compare_order(o_gpu, o_ref, mode, k, l):
    n = int(host(o_gpu["n_nodes"])[0])
    assert n == o_ref.n_nodes
    assert np.array_equal(host(o_gpu["node_heap"]), o_ref.node_heap)
    assert np.array_equal(host(o_gpu["node_vptr"]), o_ref.node_vptr)
    assert np.array_equal(host(o_gpu["vperm"]), o_ref.vperm)
    assert np.array_equal(host(o_gpu["part"]), o_ref.part)
    assert np.array_equal(host(o_gpu["split_cut"]), o_ref.split_cut)
    if mode == oracle.NET_MODE:
        assert np.array_equal(host(o_gpu["nperm"]), o_ref.nperm)
        assert np.array_equal(host(o_gpu["node_nptr"]), o_ref.node_nptr)
