"""Failure paths of the C ABI on the GPU, forced from the host so that every
kernel runs normally.

* A device allocation made to fail by the handle's test hook (TNO_FAULT=alloc:N,
  read when the handle is created: its N-th fresh allocation fails) is refused
  with TNO_E_NOMEM when nothing is in flight and TNO_E_BUSY (retry later) while
  another request holds memory; nothing is left charged and the handle serves
  the same request afterwards, matching the oracle.
* A cancelled ticket ends with TNO_E_CANCELLED, gives its memory back and can
  be neither polled nor cancelled again; the other tickets of the handle finish
  with the oracle's results, with eager launches and with batched steps.
* Destroying a handle with tickets still live drains them; a new handle works.
* A handle that reserves its budget at creation carves every buffer from it.
"""
import os

import numpy as np
import pytest
import torch

from oracle import oracle
from paper_2209_09848_amd import synth, tno
from tests import parity

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
K = 5


def _to(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _problem(seed, T=24, H=40, W=72, J=3):
    g = np.random.default_rng(seed)
    R = g.standard_normal((T, H, W)).astype(np.float32)
    sigma = (0.5 + g.random((H, W))).astype(np.float32)
    times = synth.times_uniform(T)
    vel = g.uniform(-0.3, 0.3, (J, 2))
    return R, sigma, times, vel


class _Req:
    """A request on the GPU, its outputs and the oracle's answer."""

    def __init__(self, seed, **shape):
        self.R, self.sigma, self.times, self.vel = _problem(seed, **shape)
        self.t = [_to(self.R), _to(self.sigma), _to(self.times), _to(self.vel)]
        T, H, W = self.R.shape
        self.req = tno.make_request(*self.t, t_ref=float(self.times[0]), top_k=K)
        self.o, self.out = tno.alloc_outputs(self.vel.shape[0], H, W, K, device=DEV)

    def check(self):
        torch.cuda.synchronize()
        ref = oracle.search(self.R, self.sigma, self.times, float(self.times[0]), self.vel)
        parity.check_maps(self.o["snr"].cpu().numpy(), self.o["flux"].cpu().numpy(), ref)


def _faulty_handle(n, **kw):
    os.environ["TNO_FAULT"] = "alloc:%d" % n
    try:
        return tno.Search(0, **kw)
    finally:
        del os.environ["TNO_FAULT"]


def test_forced_allocation_failure_leaves_the_handle_usable():
    a = _Req(1)
    with _faulty_handle(1) as h:
        print("allocation 1 fails, nothing in flight", flush=True)
        rc, t = tno.tno_search_submit(h.h, a.req, a.out)
        assert rc == tno.TNO_E_NOMEM and t is None
        assert "allocation" in tno.tno_search_last_error()
        st = tno.tno_search_stats(h.h)
        assert st.inflight == 0 and st.in_use_bytes == 0 and st.held_bytes == 0
        res = h.wait(h.submit(a.req, a.out))
        assert res.status == tno.TNO_OK
        a.check()
        st = tno.tno_search_stats(h.h)
        assert st.inflight == 0 and st.in_use_bytes == 0 and st.device_allocs == 2


def test_allocation_failure_with_work_in_flight_asks_for_a_retry():
    a, b = _Req(2), _Req(3)
    with _faulty_handle(2) as h:
        print("allocation 2 fails while request 1 is in flight", flush=True)
        ta = h.submit(a.req, a.out)
        rc, tb = tno.tno_search_submit(h.h, b.req, b.out)
        assert rc == tno.TNO_E_BUSY and tb is None
        assert "in flight" in tno.tno_search_last_error()
        assert h.wait(ta).status == tno.TNO_OK
        assert h.wait(h.submit(b.req, b.out)).status == tno.TNO_OK
        a.check()
        b.check()
        st = tno.tno_search_stats(h.h)
        assert st.inflight == 0 and st.in_use_bytes == 0


@pytest.mark.parametrize("batch", [False, True], ids=["eager", "batch"])
def test_cancelled_ticket_ends_cancelled_and_frees_its_memory(batch):
    reqs = [_Req(10 + i) for i in range(3)]
    with tno.Search(0, own_streams=True, batch=batch) as h:
        print("cancel the middle one of 3 tickets, batch", batch, flush=True)
        tickets = [h.submit(r.req, r.out) for r in reqs]
        assert h.cancel(tickets[1]) == tno.TNO_OK
        rc, res = tno.tno_search_poll(h.h, tickets[1], -1)
        assert rc == tno.TNO_E_CANCELLED and res.status == tno.TNO_E_CANCELLED
        rc, _ = tno.tno_search_poll(h.h, tickets[1], 0)
        assert rc == tno.TNO_E_TICKET
        assert h.cancel(tickets[1]) == tno.TNO_E_TICKET
        assert h.cancel(987654321) == tno.TNO_E_TICKET
        for i in (0, 2):
            assert h.wait(tickets[i]).status == tno.TNO_OK
            reqs[i].check()
        st = tno.tno_search_stats(h.h)
        assert st.inflight == 0 and st.in_use_bytes == 0 and st.held_bytes == 0
        # the handle keeps serving
        assert h.wait(h.submit(reqs[1].req, reqs[1].out)).status == tno.TNO_OK
        reqs[1].check()


def test_destroy_with_live_tickets_drains_them():
    reqs = [_Req(20 + i) for i in range(2)]
    print("destroy a handle with 2 live tickets", flush=True)
    h = tno.Search(0, own_streams=True)
    for r in reqs:
        h.submit(r.req, r.out)
    h.close()
    torch.cuda.synchronize()
    with tno.Search(0) as h2:
        assert h2.wait(h2.submit(reqs[0].req, reqs[0].out)).status == tno.TNO_OK
    reqs[0].check()


def test_reserved_handle_carves_its_buffers_from_one_block():
    """TNO_CFG_RESERVE: the budget is taken at creation; requests of several
    shapes run from ranges of that block with the bits of an unreserved
    handle, nothing is charged once they are collected, and a request larger
    than the block is refused."""
    reqs = [_Req(30 + i) for i in range(3)]
    with tno.Search(0) as h:
        for r in reqs:
            assert h.wait(h.submit(r.req, r.out)).status == tno.TNO_OK
    ref = [r.o["snr"].cpu().numpy().copy() for r in reqs]
    with tno.Search(0, own_streams=True, reserve=True, hbm_budget_bytes=1 << 30) as h:
        print("reserved handle, 3 requests", flush=True)
        st = tno.tno_search_stats(h.h)
        assert st.budget_bytes == 1 << 30 and st.in_use_bytes == 0
        tickets = [h.submit(r.req, r.out) for r in reqs]
        for t in tickets:
            assert h.wait(t).status == tno.TNO_OK
        for r, s in zip(reqs, ref):
            assert np.array_equal(r.o["snr"].cpu().numpy(), s)
        reqs[0].check()
        st = tno.tno_search_stats(h.h)
        assert st.inflight == 0 and st.in_use_bytes == 0 and st.cached_bytes == 0
    big = _Req(40, T=64, H=128, W=256)    # its staged stack alone is ≈ 9 MB
    with tno.Search(0, reserve=True, hbm_budget_bytes=2 << 20) as h:
        rc, t = tno.tno_search_submit(h.h, big.req, big.out)
        assert rc == tno.TNO_E_NOMEM and t is None
