"""Capture the whole pipeline in one HIP graph and replay it.

Every stage is a kernel launch on one stream with device-side list lengths,
so the sequence track -> continuation -> refine/certify -> duplicates ->
re-track rounds -> classify records into a graph once and replays without any
host round trip.  Buffers are allocated before capture and reused by every
replay; the id lists and counters are rewritten by the kernels themselves
(no memset nodes).
"""
from __future__ import annotations

import torch

from . import pipeline


class PipelineGraph:
    def __init__(self, batch: pipeline.Batch, opts: pipeline.Options,
                 bufs: pipeline.Buffers | None = None):
        self.batch, self.opts = batch, opts
        self.bufs = bufs or pipeline.allocate(batch, opts.precision)
        # one eager run loads the code objects before capture
        pipeline.run(batch, opts, self.bufs)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            pipeline.run(batch, opts, self.bufs)
        torch.cuda.synchronize()

    def replay(self) -> pipeline.Buffers:
        self.graph.replay()
        return self.bufs
