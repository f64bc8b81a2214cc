"""The Metaball-Imaging fitness without allocation (mi_fitness_noalloc)
through the C ABI, against the entry point with a caller workspace
(mi_fitness) on the same inputs: two calls in a row, the second smaller, both
spanning several chunks of hull points so that the per-chunk sums go through
the library's static scratch array.  The same kernels in the same order:
equal bit for bit.  A size beyond the scratch is refused."""
import ctypes as C

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def test_noalloc_fitness_matches_workspace_entry_point():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2209_10411_amd as mdl
    L = mdl.lib()
    dev = "cuda:0"
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    for m, P, seed in ((5000, 40, 1), (2500, 7, 2)):
        print(f"noalloc fitness m={m} P={P}", flush=True)
        cp, k = workloads.mi_body(seed=95 + seed, n_cp=6, R=8.0)
        H, pl, _ = workloads.mi_hull(cp, k, m=m)
        pop = workloads.mi_population(H, pl, P, 6, seed=97 + seed)
        ref = mdl.mi_fitness(H, pop)
        h = torch.as_tensor(H, dtype=torch.float64, device=dev)
        p = torch.as_tensor(pop, dtype=torch.float64, device=dev)
        F = torch.full((P,), float("nan"), dtype=torch.float64, device=dev)
        rc = L.mi_fitness_noalloc(C.c_void_p(h.data_ptr()), m, C.c_void_p(p.data_ptr()), P, 6,
                                  C.c_void_p(F.data_ptr()), stream)
        assert rc == 0
        torch.cuda.synchronize()
        assert np.array_equal(F.cpu().numpy(), ref)
    # 131072 chunk sums at most: 2 chunks x 70000 individuals is refused before any launch
    assert L.mi_fitness_noalloc(C.c_void_p(h.data_ptr()), 4096, C.c_void_p(p.data_ptr()), 70000, 6,
                                C.c_void_p(F.data_ptr()), stream) == -1
