"""Error paths of a device failure, forced from the host (DDKS_FAULT_INJECT, a
test-only switch read at context creation): the library acts as if the HIP
runtime had reported a launch failure at the chosen site, without launching
anything there, so no kernel faults.  Checked: a failed call poisons the
context and every later call reports DDKS_E_DEVICE; a failed serving launch
or serving event fails the tickets it held and every queued one, pollers
waiting without a timeout return, and closing the context does not hang."""
import os
import threading

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _ctx_with_fault(spec, **kw):
    from paper_2106_13706_amd import native
    old = os.environ.get("DDKS_FAULT_INJECT")
    os.environ["DDKS_FAULT_INJECT"] = spec
    try:
        return native.Context(**kw)
    finally:
        if old is None:
            os.environ.pop("DDKS_FAULT_INJECT")
        else:
            os.environ["DDKS_FAULT_INJECT"] = old


def _pair(g, n_p, n_q, d):
    return (g.standard_normal((n_p, d)).astype(np.float32),
            g.standard_normal((n_q, d)).astype(np.float32))


def _status(fn):
    from paper_2106_13706_amd import native
    try:
        fn()
    except native.DDKSError as e:
        return e.status
    return native.DDKS_OK


def test_failed_call_poisons_every_entry_point():
    import torch
    from paper_2106_13706_amd import native
    g = np.random.default_rng(1)
    P, Q = _pair(g, 300, 200, 3)
    ctx = _ctx_with_fault("call:2")
    try:
        ok = ctx.distance(P, Q)  # the first call runs normally
        with pytest.raises(native.DDKSError) as e:
            ctx.distance(P, Q)
        assert e.value.status == native.DDKS_E_DEVICE and "injected" in str(e.value)
        Pt, Qt = torch.from_numpy(P).cuda(), torch.from_numpy(Q).cuda()
        Z = np.concatenate([P, Q])
        counts = np.zeros((500, 8, 2), np.uint32)
        calls = {
            "distance": lambda: ctx.distance(P, Q),
            "distance_device": lambda: ctx.distance(Pt, Qt),
            "distance_noalloc": lambda: ctx.distance_noalloc(Pt, Qt),
            "permutation_batch": lambda: ctx.permutation_batch(Z, 300, np.zeros((0, 16), np.uint32)),
            "significance": lambda: ctx.significance(counts, 300, 200, 3, 1),
            "vdks": lambda: ctx.vdks(P, Q, 4),
            "rdks": lambda: ctx.rdks(P, Q),
            "serve_submit": lambda: ctx.serve_submit(P, Q),
        }
        for name, fn in calls.items():
            print(f"  {name}", flush=True)
            assert _status(fn) == native.DDKS_E_DEVICE, name
    finally:
        ctx.close()
    with native.Context() as fresh:  # a new context is unaffected
        assert fresh.distance(P, Q).num == ok.num


@pytest.mark.parametrize("spec", ["serve_launch:1", "serve_launch:3", "serve_event:2"])
def test_serving_failure_fails_tickets_and_drains(spec):
    """Requests go in waves of ten, each wave polled to the end by threads
    waiting without a timeout before the next is submitted, so every wave
    takes at least one launch and the failing launch or event comes by the
    third wave.  Requests of a failing launch and every one queued behind it
    end with DDKS_E_DEVICE (launches that completed before keep their
    results), every poller returns, submit then reports DDKS_E_DEVICE, and
    closing the context returns."""
    from paper_2106_13706_amd import native
    g = np.random.default_rng(2)
    reqs = [_pair(g, int(g.integers(50, 3000)), int(g.integers(50, 3000)), int(g.integers(2, 6)))
            for _ in range(60)]
    ctx = _ctx_with_fault(spec, serve_streams=2)
    done_reqs, statuses, nums = [], [], []
    try:
        for w in range(0, len(reqs), 10):
            tickets = []
            refused = False
            for P, Q in reqs[w:w + 10]:
                try:
                    tickets.append(((P, Q), ctx.serve_submit(P, Q)))
                except native.DDKSError as e:
                    assert e.status == native.DDKS_E_DEVICE
                    refused = True
                    break
            st = [None] * len(tickets)
            nm = [None] * len(tickets)

            def poll(i):
                try:
                    nm[i] = ctx.serve_poll(tickets[i][1], timeout_us=-1).num
                    st[i] = native.DDKS_OK
                except native.DDKSError as e:
                    st[i] = e.status

            threads = [threading.Thread(target=poll, args=(i,)) for i in range(len(tickets))]
            for t in threads:
                t.start()
            for t in threads:
                t.join(timeout=60)
            assert not any(t.is_alive() for t in threads), "a poller never returned"
            done_reqs += [pq for pq, _ in tickets]
            statuses += st
            nums += nm
            if refused or native.DDKS_E_DEVICE in st:
                break
        print(f"  {spec}: {statuses.count(native.DDKS_OK)} ok, "
              f"{statuses.count(native.DDKS_E_DEVICE)} failed of {len(statuses)} submitted", flush=True)
        assert set(statuses) <= {native.DDKS_OK, native.DDKS_E_DEVICE}
        assert statuses.count(native.DDKS_E_DEVICE) >= 1
        assert _status(lambda: ctx.serve_submit(*reqs[0])) == native.DDKS_E_DEVICE
        assert _status(lambda: ctx.distance(*reqs[0])) == native.DDKS_E_DEVICE
    finally:
        done = threading.Event()
        closer = threading.Thread(target=lambda: (ctx.close(), done.set()))
        closer.start()
        closer.join(timeout=60)
        assert done.is_set(), "closing the context hung"
    with native.Context() as fresh:  # results that were delivered are right
        for (P, Q), st, num in zip(done_reqs, statuses, nums):
            if st == native.DDKS_OK:
                assert fresh.distance(P, Q).num == num
