"""MI355X-native exact counting of directed pattern embeddings (XMiner's hot path).

The compute path is libxminer.so: a host planner plus gfx950 HIP kernels
behind the C ABI of include/xminer.h.  This package only marshals
arguments to it; PyTorch supplies device memory and streams.
"""
from .api import (Graph, Plan, Counter, Watchdog, count, count_anchored, describe_plan, list_embeddings,
                  plan_json, plan_traffic, plan_work, workspace_bytes)

__all__ = ["Graph", "Plan", "Counter", "Watchdog", "count", "count_anchored", "describe_plan",
           "list_embeddings", "plan_json", "plan_traffic", "plan_work", "workspace_bytes"]
