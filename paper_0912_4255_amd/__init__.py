"""MI355X-native barycentric-resampling F-statistic (arXiv:0912.4255).

The hot path (resampling, FFTs, F-statistic, gradients) runs in HIP kernels
for gfx950 inside librsfstat.so, reached through the C ABI declared in
include/rsfstat.h.  This package is the thin Python binding.
"""
from ._lib import (RSF_ENTRY_BACKWARD, RSF_ENTRY_FSTAT, RSF_ENTRY_POINT, RSF_ENTRY_RESAMPLE,
                   RSF_ENTRY_SEMICOHERENT, RSF_ENTRY_TOPK,
                   RSF_FLAG_DEGENERATE, RSF_FLAG_ORBIT, RSF_FLAG_WINDOW, RSF_MODE_BATCHED, RSF_MODE_PLAIN, RsfError,
                   load)


def __getattr__(name):
    # torch is imported lazily so that the pure-Python parts (synth, build)
    # work without it
    if name in ("Plan", "plan_desc_from_workload", "FStatFn", "fstat_point", "SftPlan", "sft_desc_from_set", "HetdecPlan",
                "fstat_topk_segments", "graph_topk_segments", "segments_workspace"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
