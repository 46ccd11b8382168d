"""Drives the request server's scheduler (tests/host/server_mock.cpp built as a
shared library) from Python with the device-memory hook set to Python
callbacks, as a framework's caching allocator would be: every setup worker and
the driver thread then allocate and free through ctypes callbacks.

usage: python server_callbacks_driver.py <mock .so> <rounds> <fail_every>
Prints "OK ..." when every request came back with the outputs of its own
ticket, every block handed out was handed back and no handle is left.
"""
import ctypes as C
import gc
import math
import os
import random
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from paper_1901_02090_amd import bddc as B  # noqa: E402


def main():
    lib = C.CDLL(sys.argv[1])
    rounds, fail_every = int(sys.argv[2]), int(sys.argv[3])
    P = C.c_void_p
    lib.bddc_set_allocator.argtypes = [B.ALLOC_FN, B.FREE_FN, C.c_void_p]
    lib.bddc_server_create.argtypes = [C.POINTER(B.ServerOptions), C.POINTER(P)]
    lib.bddc_server_submit.argtypes = [P, C.POINTER(B.Request), C.POINTER(C.c_uint64)]
    lib.bddc_server_poll.argtypes = [P, C.c_uint64, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                     C.POINTER(B.RequestStats)]
    lib.bddc_server_stats.argtypes = [P, C.POINTER(B.ServerStats)]
    lib.bddc_server_destroy.argtypes = [P]
    lib.bddc_last_error.restype = C.c_char_p
    lib.mock_live_handles.restype = C.c_long
    lib.mock_live_blocks.restype = C.c_long

    live, lock, calls = {}, threading.Lock(), [0, 0, 0]
    rng = random.Random(7)

    def alloc(n, ctx):
        # interpreter work on the calling (native) thread: garbage, a collection now and then
        with lock:
            calls[0] += 1
            k = calls[0]
        junk = [bytearray(64) for _ in range(16)]
        if k % 11 == 0:
            gc.collect()
        if fail_every and k % fail_every == 0:
            calls[2] += 1
            return None                       # the caller's allocator has no memory
        buf = C.create_string_buffer(int(n))
        addr = C.addressof(buf)
        with lock:
            live[addr] = buf
        del junk
        return addr

    def free(p, ctx):
        with lock:
            calls[1] += 1
            live.pop(p)
        if rng.random() < 0.05:
            time.sleep(0.0005)

    a, f = B.ALLOC_FN(alloc), B.FREE_FN(free)
    assert lib.bddc_set_allocator(a, f, None) == 0
    bad = 0
    for rnd in range(rounds):
        opt = B.ServerOptions(0.0, 4, 2, B.BDDC_MIXED, 0)
        h = P()
        assert lib.bddc_server_create(C.byref(opt), C.byref(h)) == 0
        reqs = [W.serving_request(rnd * 1000 + k) for k in range(48)]
        tickets, keep = [], []
        for pr in reqs:
            g, part, cuts = B._grid_part(pr.n, pr.h, pr.cuts)
            perm = np.ascontiguousarray(pr.perm, dtype=np.float64).reshape(-1)
            src = np.ascontiguousarray(pr.source, dtype=np.float64)
            rq = B.Request(g, B._dptr(perm), part, B._tau(pr.tau), B._dptr(src), 1e-8, 0)
            t = C.c_uint64()
            assert lib.bddc_server_submit(h, C.byref(rq), C.byref(t)) == 0, lib.bddc_last_error()
            tickets.append(t.value)
            keep.append((src, pr))
            time.sleep(rng.random() * 0.002)
        if rnd % 3 == 2:
            lib.bddc_server_destroy(h)             # requests still in flight
            continue
        n_ok = n_fail = 0
        for t, (src, pr) in zip(tickets, keep):
            nc = int(np.prod(pr.n))
            nn = list(pr.n) + [1] * (3 - len(pr.n))
            nf = sum(int(np.prod([nn[e] + (e == d) for e in range(3)])) for d in range(len(pr.n)))
            flux, pres = np.full(nf, -1.0), np.full(nc, -1.0)
            st = B.RequestStats()
            rc = lib.bddc_server_poll(h, t, -1.0, B._dptr(flux), B._dptr(pres), C.byref(st))
            if rc == 0:
                n_ok += 1
                if not (np.array_equal(flux, np.arange(nf) + nc) and np.array_equal(pres, 2.0 * src)):
                    print(f"FAIL round {rnd} ticket {t}: outputs of another request")
                    bad += 1
            elif rc == B.BDDC_ENOMEM and fail_every:
                n_fail += 1
            else:
                print(f"FAIL round {rnd} ticket {t}: rc {rc} {lib.bddc_last_error().decode()}")
                bad += 1
        ss = B.ServerStats()
        lib.bddc_server_stats(h, C.byref(ss))
        if ss.completed + ss.failed != len(tickets):
            bad += 1
        lib.bddc_server_destroy(h)
        print(f"round {rnd}: {n_ok} solved, {n_fail} out of memory", flush=True)
    if lib.mock_live_handles() != 0 or lib.mock_live_blocks() != 0 or live:
        print(f"FAIL handles {lib.mock_live_handles()} blocks {lib.mock_live_blocks()} python {len(live)}")
        bad += 1
    print(f"{'FAIL' if bad else 'OK'} rounds {rounds} allocations {calls[0]} frees {calls[1]} refused {calls[2]}",
          flush=True)
    return 1 if bad else 0


if __name__ == "__main__":
    sys.exit(main())
