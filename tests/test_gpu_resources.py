"""Resource lifetime of the library's per-thread caches: host threads that fit
on their own streams hand their device memory back when they exit (freed by
the next call on any thread, so thread generations do not add up), and
ms_release_workspace frees what the calling thread holds."""
import ctypes
import sys
import threading

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2112_13891_amd import api, workloads  # noqa: E402

DEV = "cuda:0"
SLACK = 4 << 20   # bytes of device memory the runtime may keep for itself


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _free_bytes():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return torch.cuda.mem_get_info()[0]


def _fit_raw(X, modes, labels, h, precision, stream):
    """ms_fit through the C ABI on caller buffers and a caller stream, so that
    the only device memory the calling thread allocates is the library's."""
    p = api.make_params(h, precision=precision)
    k = ctypes.c_int32(0)
    dg = api.Diag()
    rc = api.lib().ms_fit(ctypes.byref(p), ctypes.c_void_p(X.data_ptr()), X.shape[0], X.shape[1],
                          ctypes.c_void_p(modes.data_ptr()), modes.shape[0], ctypes.byref(k),
                          ctypes.c_void_p(labels.data_ptr()), ctypes.byref(dg),
                          ctypes.c_void_p(stream.cuda_stream))
    return rc, int(k.value), int(dg.workspace_bytes)


def test_exited_threads_leave_no_device_memory():
    X = workloads.aniso3d(seed=0).X
    nt = 4
    # every tensor and stream is made here, on the main thread
    Xs = [torch.from_numpy(X[i * 10_000:]).to(DEV) for i in range(nt)]
    modes = [torch.empty((len(x), 3), dtype=torch.float32, device=DEV) for x in Xs]
    labels = [torch.empty(len(x), dtype=torch.int32, device=DEV) for x in Xs]
    streams = [torch.cuda.Stream(device=DEV) for _ in range(nt)]
    held = []

    def work(i, errors):
        try:
            rc, k, ws = _fit_raw(Xs[i], modes[i], labels[i], 15.0, 1 if i % 2 else 0, streams[i])
            assert rc == 0 and k > 0, (rc, api.last_error())
            held.append(ws)
        except Exception as e:   # reported by the main thread
            errors.append(repr(e))

    def round_of_threads():
        errors = []
        threads = [threading.Thread(target=work, args=(i, errors)) for i in range(nt)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        assert not errors, errors

    # a first generation brings up whatever the runtime keeps per process
    round_of_threads()
    api.release_workspace()
    base = _free_bytes()
    # threads exit holding their caches; the next call on any thread frees
    # them, so generations of threads do not add up: a leak would take a
    # whole generation's caches more each time.  (The HIP runtime itself
    # keeps a few tens of MiB per exited host thread for a while, more or
    # less from one generation to the next; half a generation's caches
    # bounds that noise.)
    free = []
    for g in range(4):
        held.clear()
        round_of_threads()
        free.append(_free_bytes())
    generation = sum(held)
    growth = max(free[0] - f for f in free[1:])
    say("device workspace held by one generation", held, "free at baseline", base, "after each generation",
        free, "largest growth", growth)
    assert generation > 4 * SLACK   # enough held that a leak would show
    assert growth <= generation // 2, (growth, generation)
    # and nothing stays once the exited threads' caches are released
    api.release_workspace()
    after = _free_bytes()
    assert base - after <= generation // 2, (base - after, generation)


def test_release_workspace_frees_calling_thread_cache():
    X = torch.from_numpy(workloads.aniso3d(seed=0).X).to(DEV)
    api.fit(X, 15.0, precision="bf16")
    held = _free_bytes()
    api.release_workspace()
    freed = _free_bytes()
    say("released", freed - held, "bytes")
    assert freed - held > SLACK
    # the next call allocates again and gives the same result
    a = api.fit(X, 15.0, precision="bf16", trace=True)
    api.release_workspace()
    b = api.fit(X, 15.0, precision="bf16", trace=True)
    assert torch.equal(a.modes, b.modes) and torch.equal(a.labels, b.labels)
