"""G-SP2 density matrices on AMD Instinct MI355X: Python binding of libgsp2.so.

The computation lives in the HIP library (include/gsp2.h); this package only
marshals arguments.  See ``gsp2`` for the calls, which keep the C names.
"""
from .gsp2 import (DeviceCSR, Gsp2Error, Plan, csr_to_device, gsp2_backward, gsp2_core_halo_host, gsp2_density,
                   gsp2_density_noalloc, gsp2_locality_graph, gsp2_partition_anneal, gsp2_plan_create, gsp2_plan_destroy, gsp2_plan_graph,
                   gsp2_plan_tune, gsp2_probe_mfma, gsp2_plan_part_index, gsp2_plan_pattern, gsp2_plan_query, gsp2_plan_set_stream,
                   gsp2_run_options_default, gsp2_run_status, gsp2_run_timing, gsp2_sparse_sp2_host, load, LIB_PATH,
                   STATUS_NAMES)

__all__ = [
    "DeviceCSR", "Gsp2Error", "Plan", "csr_to_device", "gsp2_backward", "gsp2_core_halo_host", "gsp2_density",
    "gsp2_density_noalloc", "gsp2_locality_graph", "gsp2_partition_anneal", "gsp2_plan_create", "gsp2_plan_destroy", "gsp2_plan_graph",
    "gsp2_plan_tune", "gsp2_probe_mfma", "gsp2_plan_part_index", "gsp2_plan_pattern", "gsp2_plan_query", "gsp2_plan_set_stream",
    "gsp2_run_options_default", "gsp2_run_status", "gsp2_run_timing", "gsp2_sparse_sp2_host",
    "load", "LIB_PATH", "STATUS_NAMES",
]
