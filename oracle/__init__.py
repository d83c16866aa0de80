"""Oracle for the gemm library: plain, slow, obviously correct CPU code.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It shares no code
with the GPU library and never imports it; inputs reach it as numpy/torch CPU
arrays produced by the seeded generators.

Contents
  gemm            FP64 C = alpha*A*B + beta*C0 (Tiramisu paper, Section I,
                  the gemm problem statement) via liboracle.so (gemm_ref.c).
  precision       bf16 / e4m3 rounding, the split-bf16x3 expected value and
                  the per-tile quantiser (project precision forms; their
                  readings are stated in each function).
  normwise_error  ||X - R||_F / ||R||_F in FP64.
  mlp             FP64 ReLU MLP, MSE loss, chain-rule gradients and Adam
                  (the cost model's network).
  conv            FP64 R x R 'same' convolution layer, NHWC (the Conv layer
                  of Section VI-A as an implicit gemm's reference).
  gemm2           FP64 back-to-back gemm alpha * act(A B) D + beta * E0
                  (the fused layer pair of Section VI-A's VGG block).
  contract        FP64 binary tensor contraction over labelled modes (the
                  Baryon benchmark's operation, Section VI-A).
"""
from .gemm import gemm, gemm_rows, num_threads, normwise_error, lib_path  # noqa: F401
from . import precision  # noqa: F401
from . import mlp  # noqa: F401
from . import conv  # noqa: F401
from . import gemm2  # noqa: F401
from . import contract  # noqa: F401
