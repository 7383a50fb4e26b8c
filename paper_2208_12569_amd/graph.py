"""Q maps captured into a HIP graph.

fastqsl_q2d allocates nothing, synchronises nothing and clears its workspace with a
fill kernel (no memset node), so a whole call, batched jobs included, can be
captured once and replayed. The graph keeps the device addresses it was captured
with: the field tensors must stay alive and be updated in place between replays,
and every replay overwrites the same output tensors.
"""

from __future__ import annotations

from typing import Optional, Sequence

from . import Params, _torch, alloc_q2d_outputs, q2d_batch_into, q2d_workspace_size


class Q2DGraph:
    """One persistent-launch batch of q2d maps, captured once and replayed."""

    def __init__(self, jobs: Sequence, params: Optional[Params] = None, want_lines: bool = False):
        torch = _torch()
        self.jobs = list(jobs)
        self.params = params or Params()
        if self.params.events is not None:
            raise ValueError("timing events cannot be recorded inside a captured graph")
        dev = self.jobs[0][0].device
        need = q2d_workspace_size(self.jobs, self.params)
        self.ws = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
        self.outs = alloc_q2d_outputs(self.jobs, want_lines)
        # one eager run on a side stream first (loads the code objects, as torch
        # asks before capture)
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            q2d_batch_into(self.jobs, self.outs, self.ws, self.params)
        torch.cuda.current_stream(dev).wait_stream(side)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            q2d_batch_into(self.jobs, self.outs, self.ws, self.params)

    def replay(self) -> list:
        """Run the captured call on the current stream; returns the output maps."""
        self.graph.replay()
        return self.outs
