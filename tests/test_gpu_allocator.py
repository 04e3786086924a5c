"""Device memory through the caller's allocator (pico_set_allocator, bound to
torch's caching allocator): every workspace of pico_init, pico_init_reduced,
pico_pmr_cs and the serving budget is taken from it, returned to it, and the
results are unchanged.
"""
import sys

import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    from paper_2605_09590_amd import pico as lib
    lib.load()
    assert torch.cuda.is_available()
    yield lib
    lib.pico_set_allocator()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


class Counting:
    """torch caching-allocator callbacks that log live blocks."""

    def __init__(self):
        self.live = {}
        self.calls = 0

    def alloc(self, n):
        p = torch.cuda.caching_allocator_alloc(n)
        self.live[p] = n
        self.calls += 1
        return p

    def free(self, p):
        self.live.pop(p)
        torch.cuda.caching_allocator_delete(p)


def _round512(n):
    return (n + 511) // 512 * 512


def _phase_encode(lib, seed=0):
    prob = workloads.config(1, seed=seed, probes=8, cg_iters=20)
    maps = _dev(prob.maps.astype(np.complex64))
    mask = _dev(prob.mask)
    return prob, maps, mask


def test_torch_allocator_holds_every_operator_byte(lib):
    say("case: pico_set_allocator -> torch caching allocator, 64x64 4-coil phase-encode op, 8 probes")
    prob, maps, mask = _phase_encode(lib)
    n = prob.ny * prob.nx
    # reference map with hipMalloc workspaces
    lib.pico_set_allocator()
    h0 = lib.pico_init(prob.ny, prob.nx, maps, prob.psi, mask, cg_iters=20, probe_tile=8, lam=0.05)
    s0 = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    lib.pico_noise_map(h0, 11, 0, 8, 0, lib.make_accum(s0))
    torch.cuda.synchronize()
    lib.pico_destroy(h0)

    cnt = Counting()
    lib.pico_set_allocator(cnt.alloc, cnt.free)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    h = lib.pico_init(prob.ny, prob.nx, maps, prob.psi, mask, cg_iters=20, probe_tile=8, lam=0.05)
    resident, peak = lib.pico_op_bytes(h)
    assert cnt.calls > 10
    assert sum(cnt.live.values()) == resident           # every resident byte came from torch
    assert torch.cuda.memory_allocated() - base == sum(_round512(v) for v in cnt.live.values())
    s1 = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    lib.pico_noise_map(h, 11, 0, 8, 0, lib.make_accum(s1))
    torch.cuda.synchronize()
    assert torch.equal(s0, s1)                          # same kernels, same result
    del s1
    lib.pico_destroy(h)
    assert cnt.live == {}
    assert torch.cuda.memory_allocated() == base
    say(f"  resident {resident} B in {cnt.calls} blocks (peak {peak} B), all returned")

    # the reduced-grid temporaries and operator go through it too (128^2 -> 64^2)
    rng = np.random.default_rng(4)
    maps2 = _dev(workloads.coil_maps(128, 128, 4, rng).astype(np.complex64))
    psi2 = workloads.noise_cov(4, rng)
    mask2 = _dev(workloads.cart_mask_1d(128, 2, 8))
    calls = cnt.calls
    hr = lib.pico_init_reduced(2, 128, 128, maps2, psi2, mask2, cg_iters=20, probe_tile=8)
    r_res, _ = lib.pico_op_bytes(hr)
    assert cnt.calls > calls and sum(cnt.live.values()) == r_res
    lib.pico_destroy(hr)
    assert cnt.live == {}

    # a server's budget is one block from it
    srv = lib.pico_server_create(64 << 20, 2, 2)
    assert list(cnt.live.values()) == [64 << 20]
    lib.pico_server_destroy(srv)
    assert cnt.live == {}
    lib.pico_set_allocator()


def test_allocator_failure_is_enomem_and_leaks_nothing(lib):
    say("case: allocator that fails after 5 blocks -> PICO_ENOMEM, every block returned")
    prob, maps, mask = _phase_encode(lib, seed=1)
    cnt = Counting()
    budget = {"left": 5}

    def alloc(n):
        if budget["left"] == 0:
            return 0
        budget["left"] -= 1
        return cnt.alloc(n)

    lib.pico_set_allocator(alloc, cnt.free)
    with pytest.raises(lib.PicoError) as ei:
        lib.pico_init(prob.ny, prob.nx, maps, prob.psi, mask, cg_iters=20, probe_tile=8)
    assert ei.value.status == lib.PICO_ENOMEM
    assert cnt.calls == 5 and cnt.live == {}
    lib.pico_set_allocator()
