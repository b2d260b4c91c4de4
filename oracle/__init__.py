"""CPU oracle for the RTL-simulation cascade (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The GPU library does not depend on it in any way.
"""
from .levelize import NotLevelizable, layer_order, levelize
from .fuse import fuse_mux_chains, mux_links
from .oracle import build, eval_op, lib_path, run, splitmix64, stim

__all__ = ["build", "eval_op", "lib_path", "run", "splitmix64", "stim", "levelize",
           "layer_order", "NotLevelizable", "fuse_mux_chains", "mux_links"]
