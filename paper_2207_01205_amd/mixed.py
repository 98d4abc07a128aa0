"""Blocks of several geometries extrapolated together.

A ``MixedBatch`` holds one plan per geometry (area size, FFT size, K, missing
area).  ``extrapolate`` starts every class on its own HIP stream, forked from
the caller's stream and joined back to it with events, so the kernels of the
classes run concurrently and a graph captured on the caller's stream holds the
whole mixed batch as one launch.  All arithmetic is in the classes' kernels.
"""

from __future__ import annotations


class MixedBatch:
    """Call ``extrapolate`` once outside a graph capture before capturing it
    (plan-owned buffers are allocated on first use)."""

    def __init__(self, plans):
        import torch
        self.plans = list(plans)
        self.device = self.plans[0].device
        dev = torch.device("cuda", self.device)
        self.streams = [torch.cuda.Stream(dev) for _ in self.plans]

    def extrapolate(self, inputs, rho_gamma, outs, records=None, statuses=None, concurrent=True):
        """inputs[c] = (areas, known or None) of class c; outs[c] its output
        tensor [n_c, nB_c]; records[c] = (sel, coef) or None; statuses[c] a
        status tensor or None.  Enqueued on the current stream (classes on
        forked streams when ``concurrent``)."""
        import torch
        from . import fofse as F
        dev = torch.device("cuda", self.device)
        main = torch.cuda.current_stream(dev)
        for c, plan in enumerate(self.plans):
            areas, known = inputs[c]
            sel, coef = records[c] if records is not None and records[c] is not None else (None, None)
            st = statuses[c] if statuses is not None else None
            s = self.streams[c] if concurrent else main
            if concurrent:
                s.wait_stream(main)
            with torch.cuda.stream(s):
                F.fofse_extrapolate_batch(plan.handle, int(areas.shape[0]), areas.data_ptr(),
                                          known.data_ptr() if known is not None else 0,
                                          rho_gamma.data_ptr(), outs[c].data_ptr(),
                                          sel.data_ptr() if sel is not None else 0,
                                          coef.data_ptr() if coef is not None else 0,
                                          st.data_ptr() if st is not None else 0, s.cuda_stream)
        if concurrent:
            for s in self.streams:
                main.wait_stream(s)
