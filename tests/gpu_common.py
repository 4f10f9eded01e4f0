"""Shared helpers of the GPU parity tests (inputs from workloads/, expected
values from oracle/)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1803_09876_amd as J  # noqa: E402
import workloads as W  # noqa: E402


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    J.load_library()


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def gpu_graph(problem, flags=0):
    return J.build_graph(problem.mesh, problem.omega, problem.weight, flags)


def rel_max(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
