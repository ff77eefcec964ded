"""The oracle schedule that a GPU solve follows cycle by cycle.

DI-SOP on the window push runs its configured rounds over each tile (two by
default: the oracle's TILED schedule with the graph's tile and a near reach
of 512 ids); the pull, the push, DI-CYC and PI run the frontier-synchronous
cycle (SYNC).
"""

import oracle
from paper_1204_6255_amd import di

REACH = 512  # near links of the window push: |i - j| <= REACH


def schedule_of(g, kernel, method=di.DI_SOP):
    """(schedule, keyword arguments) for oracle.diter / oracle.di_cycle that
    mirror a GPU solve with `kernel` on graph g (for DI_KERNEL_AUTO, once the
    graph's first such solve has tuned it)."""
    if method != di.DI_SOP:
        return oracle.SYNC, {}
    t = di.di_graph_tuning(g.handle)
    window = kernel == di.DI_KERNEL_WINDOW or (kernel == di.DI_KERNEL_AUTO and t["kernel"] == "window")
    if window and t["rounds"] == 2:
        return oracle.TILED, dict(tile=t["tile"], reach=REACH, rounds=2)
    return oracle.SYNC, {}
