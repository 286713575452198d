"""Friedkin-Johnsen equilibrium z = (I+L)^{-1} s by residual push with
over-relaxation (arXiv 2507.14864) on MI355X: a C-ABI HIP library (libfj.so,
include/fj.h) and its Python binding."""
from .fj import (Batch, FJError, FJNotConverged, Graph, certify, jacobi_steps, lib, metrics, metrics_bounds, solve,  # noqa: F401
                 metrics_noalloc, metrics_noalloc_bytes, gather_probe, batch_tune_cache_clear,
                 estimate_omega, optimal_omega, stress, tune_omega, wsnet_forward, wsnet_forward_timed, wsnet_grad, wsnet_param_count,
                 wsnet_train_step)

__all__ = ["Graph", "Batch", "solve", "metrics", "metrics_bounds", "metrics_noalloc", "metrics_noalloc_bytes", "gather_probe", "batch_tune_cache_clear", "stress", "certify", "estimate_omega", "optimal_omega", "tune_omega", "lib", "FJError", "FJNotConverged", "jacobi_steps",
           "wsnet_forward", "wsnet_forward_timed", "wsnet_grad", "wsnet_param_count", "wsnet_train_step"]
