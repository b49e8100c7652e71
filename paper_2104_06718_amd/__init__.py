"""MI355X (gfx950) Lagrangian-decomposition bounding step.

Python binding of the C ABI in include/ld.h: ``Net``, ``Batch``, ``State``,
``init_duals``, ``dual_eval`` (``dual_eval_f64``), ``step``, ``prox_step`` and
``final_bound`` call the HIP library directly; ``LDDual`` wraps ``dual_eval`` as a
torch.autograd.Function.
"""
from .binding import (Batch, LDDual, LDError, Net, State, TAU_DEFAULT, dual_eval, dual_eval_f64,  # noqa: F401
                      dual_eval_noalloc, rounding_margin,
                      final_bound, bab, branch_children, fsb_branch, init_duals, intermediate_bounds, ld_dual,
                      load_library, profile_iteration, prox_profile_iteration, prox_step, sigmoid_hull,
                      sigmoid_inner_min, set_validation, step, autotune, tuning_info, tile_candidates,
                      set_tuned_config,
                      LD_OK, LD_E_ARG, LD_E_SHAPE, LD_E_NUMERIC, LD_E_NOMEM, LD_E_DEVICE, LD_E_UNSUPPORTED,
                      LD_E_STATE, LD_FP32, LD_BF16, LD_FP64)
