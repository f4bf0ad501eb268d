"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This package only draws input data: graphs in forward CSR form, per-edge
probabilities encoded as uint32 thresholds, query seed sets and request
arrival times.  It holds none of the influence method's arithmetic (no ranks,
no live-edge coins, no reachability, no estimators); both the HIP library and
the CPU oracle receive exactly these arrays.

Probability encoding used everywhere: an edge with probability p carries
thr = floor((2^32 - 1) * p); for p = 1/d this is (2^32 - 1) // d.
"""
from .graphs import (  # noqa: F401
    Graph,
    er_graph,
    chung_lu_graph,
    rmat_graph,
    from_edges,
    uniform_thresholds,
    wc_thresholds,
    trivalency_thresholds,
)
from .queries import (  # noqa: F401
    lognormal_query_sets,
    neighbourhood_query_sets,
    poisson_arrivals,
    uniform_query_sets,
)
from .configs import CONFIGS, make_config  # noqa: F401
