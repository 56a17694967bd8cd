"""Streaming of the trajectory output off the device, overlapped with integration.

The paper writes (tau, t, x, y, z) of every particle at every step from the host
(Section 5), and most of its run time went there.  Here the kernel writes decimated
records into a device buffer (``integrate_record``) and this driver moves them to
the host while the next chunk of steps runs:

- two device record buffers and two pinned host buffers (double buffering);
- chunk k integrates into device buffer k % 2 on the caller's stream;
- a second stream (default priority) copies it to pinned host buffer k % 2 once
  the chunk's kernel has finished, while chunk k + 1 integrates;
- a writer thread hands each host buffer to ``sink`` once its copy has completed,
  and releases it for chunk k + 2.

Chunk k + 2 reuses device buffer k % 2 only after the copy of chunk k has finished
(the compute stream waits on that copy's event), and host buffer k % 2 only after
the sink has returned.
"""
import queue
import threading
from typing import Callable, Optional

import numpy as np
import torch

from . import integrate_record


class FileSink:
    """Appends each chunk's records to a binary file: float64, C order, shape
    [records, 5, n] over the whole run, k = (tau, t, x, y, z)."""

    def __init__(self, path: str):
        self.f = open(path, "wb")
        self.records = 0

    def __call__(self, recs: np.ndarray, chunk: int):
        self.f.write(memoryview(np.ascontiguousarray(recs)).cast("B"))
        self.records += recs.shape[0]

    def close(self):
        self.f.close()


def stream_trajectories(state: torch.Tensor, status: torch.Tensor, steps: torch.Tensor, spacetimes,
                        h: float, n_steps: int, record_every: int, records_per_chunk: int,
                        sink: Callable[[np.ndarray, int], None], st_of_lane=None,
                        formulation: str = "christoffel", horizon_factor: float = 1.01,
                        r_escape: float = 1500.0, block: int = 0,
                        copy_stream: Optional[torch.cuda.Stream] = None) -> dict:
    """Integrate n_steps in chunks of records_per_chunk * record_every steps and pass
    every chunk's records (a host array [records, 5, n]) to sink(records, chunk) in
    order.  Returns counts of chunks and bytes moved."""
    if record_every < 1 or records_per_chunk < 1 or n_steps % record_every:
        raise ValueError("n_steps must be a multiple of record_every >= 1")
    n = state.shape[-1]
    n_rec = n_steps // record_every
    R = min(records_per_chunk, max(n_rec, 1))
    dev = [torch.empty((R, 5, n), dtype=torch.float64, device=state.device) for _ in range(2)]
    host = [torch.empty((R, 5, n), dtype=torch.float64, pin_memory=True) for _ in range(2)]
    computed = [torch.cuda.Event() for _ in range(2)]
    copied = [torch.cuda.Event() for _ in range(2)]
    host_free = [threading.Event() for _ in range(2)]
    for e in host_free:
        e.set()
    compute = torch.cuda.current_stream()
    copy = copy_stream if copy_stream is not None else torch.cuda.Stream()
    work: "queue.Queue" = queue.Queue()
    errors = []

    def writer():
        while True:
            item = work.get()
            if item is None:
                return
            j, k, nr = item
            try:
                copied[j].synchronize()
                if not errors:
                    sink(host[j][:nr].numpy(), k)
            except Exception as exc:  # reported after the loop
                errors.append(exc)
            finally:
                host_free[j].set()

    th = threading.Thread(target=writer, daemon=True)
    th.start()
    chunks, done = 0, 0
    try:
        while done < n_rec:
            j = chunks % 2
            nr = min(R, n_rec - done)
            if chunks >= 2:
                compute.wait_event(copied[j])  # the copy of chunk k - 2 left dev[j]
            integrate_record(state, status, steps, spacetimes, h, nr * record_every, record_every,
                             traj=dev[j][:nr], horizon_factor=horizon_factor, r_escape=r_escape,
                             block=block, st_of_lane=st_of_lane, formulation=formulation)
            computed[j].record(compute)
            host_free[j].wait()  # the sink has returned host[j] of chunk k - 2
            host_free[j].clear()
            with torch.cuda.stream(copy):
                copy.wait_event(computed[j])
                host[j][:nr].copy_(dev[j][:nr], non_blocking=True)
                copied[j].record(copy)
            work.put((j, chunks, nr))
            done += nr
            chunks += 1
    finally:
        work.put(None)
        th.join()
    compute.wait_stream(copy)
    if errors:
        raise errors[0]
    return {"chunks": chunks, "records": n_rec, "bytes": n_rec * 5 * n * 8}
