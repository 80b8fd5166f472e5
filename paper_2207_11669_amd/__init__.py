"""DCF-PCA (arXiv 2207.11669) on one MI355X: the HIP library librpca.so and
its ctypes binding. See include/rpca.h for the C ABI."""
from .binding import (DCFPCA, RpcaError, colmajor, declared_functions, load_library,  # noqa: F401
                      make_params, mlp_forward, mlp_param_count, mlp_train_step, params_error,
                      workspace_bytes)
