"""librtdetmcd: RT-DetMCD (arXiv 1910.05615) with hand-written HIP kernels for MI355X.

The compute path is the in-tree shared library ``librtdetmcd.so`` (C ABI in
``include/rtdetmcd.h``); this package only marshals arguments to it.
"""
from .api import (Fit, RobustMCD, RTDetMCDError, backward, chi2_cdf, chi2_quantile,  # noqa: F401
                  consistency, cstep, distances, distances_into, fit, fit_batched, make_opts, plan, score,
                  random_partition, score_into, select, sort_reruns, START_WARM, profile,
                  profile_read, tuned_plans)
