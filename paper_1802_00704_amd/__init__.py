"""MI355X-native third-order gas-kinetic scheme on triangle meshes.

The compute path is the HIP library ``libgks.so`` (C ABI in include/gks.h);
this package is its thin Python binding.  Importing it does not load the
library; the first call does, and raises if it has not been built.
"""
from ._lib import (GKS_FP64, GKS_INNER_GMRES, GKS_INNER_RICHARDSON, GKS_MIXED, GKS_ORDER_MULTICOLOR, GKS_ORDER_RCM,
                   LIMIT_CHARACTERISTIC,
                   LIMIT_CONSERVATIVE, GksBatch, GksError, GksMesh, NonConvergence, NonPhysical, default_params,
                   host_inspect, lib)

__all__ = ["GksMesh", "GksBatch", "GksError", "NonConvergence", "NonPhysical", "default_params", "host_inspect", "lib",
           "GKS_FP64", "GKS_MIXED", "GKS_ORDER_MULTICOLOR", "GKS_ORDER_RCM", "LIMIT_CONSERVATIVE",
           "LIMIT_CHARACTERISTIC", "GKS_INNER_RICHARDSON", "GKS_INNER_GMRES"]
