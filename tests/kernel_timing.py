"""Isolated timings of the block-product shapes and of the batched LU (GPU only; not a test).

Runs the test-only kernel harness librgf_ktest.so (built by build()) on the
shapes that make up one layer of the C4 sweep (Mp = 1024, 64 energies per
launch) and on the skinny products of the KPM solve sweeps, and prints
microseconds and TFLOP/s per shape (8 real flops per complex multiply-add).
With --sweep-variants it times the two sweep products with the operand forms
the sweep uses (formed, adjoint-formed or stored), FP64 and FP32.
With --fp32 the shapes and the LU run on the FP32 matrix cores (the mixed form).
Usage: python tests/kernel_timing.py [--only-product | --sweep-variants] [--fp32]
"""
import ctypes as C
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SHAPES = [  # (tile, rows, cols, K, batch, in place, label)
    (128, 960, 960, 64, 64, 0, "LU trailing update at k0 = 0: 960 x 960, K = 64"),
    (128, 896, 896, 128, 64, 0, "the same shape class with K = 128 (896 x 896)"),
    (128, 64, 1024, 64, 64, 1, "U12 / solve diagonal block: 64 x 1024, K = 64, in place"),
    (64, 64, 1024, 64, 64, 1, "the same with 64 x 64 tiles"),
    (128, 64, 1024, 128, 64, 0, "64-row product with K = 128: 64 x 1024"),
    (64, 64, 1024, 128, 64, 0, "the same with 64 x 64 tiles"),
    (128, 128, 1024, 512, 64, 0, "solve update: 128 x 1024, K = 512"),
    (128, 128, 1024, 896, 64, 0, "solve update: 128 x 1024, K = 896"),
    (128, 1024, 1024, 1024, 64, 0, "sweep product: 1024 x 1024, K = 1024"),
    (64, 1024, 64, 1024, 1, 0, "one unsplit KPM sweep step: 1024 x 64, K = 1024, batch 1"),
    (64, 1024, 64, 64, 16, 0, "the same step as 16 chunks of K = 64 in one launch"),
    (64, 1024, 64, 1024, 400, 0, "KPM layer-batched product: 1024 x 64, K = 1024, batch 400"),
]


def main():
    import torch
    lib = C.CDLL(os.path.join(ROOT, "paper_2609_37058_amd", "librgf_ktest.so"))
    lib.rgf_ktest_gemm_time.argtypes = [C.c_int] * 8 + [C.POINTER(C.c_double)]
    lib.rgf_ktest_lu_time.argtypes = [C.c_int] * 5 + [C.POINTER(C.c_double)] * 2
    lib.rgf_ktest_sweep_time.argtypes = [C.c_int] * 5 + [C.POINTER(C.c_double)]
    torch.cuda.init()
    ms = C.c_double()
    if "--sweep-variants" in sys.argv:
        names = ["W' = -W X, stored operands", "B' = A - L X, L adjoint-formed, A formed",
                 "B' with L stored, A formed", "B' with L formed untransposed", "-L X, L adjoint-formed, no C",
                 "adjoint formation kernel + B' with L stored"]
        cases = [(Mp, nb, prec, v) for Mp, nb in ((1024, 64), (512, 64), (256, 128)) for prec in (0, 1)
                 for v in range(len(names)) if Mp == 1024 or v in (0, 1, 5)]
        for Mp, nb, prec, v in cases:
            rc = lib.rgf_ktest_sweep_time(prec, v, Mp, nb, 5, C.byref(ms))
            fl = 8.0 * Mp ** 3 * nb
            print(f"| Mp={Mp} x {nb} | {'FP64' if prec == 0 else 'FP32'} | {names[v]} | {ms.value:.3f} ms | "
                  f"{fl / ms.value / 1e9:.1f} TFLOP/s | rc={rc}", flush=True)
        return
    shapes = SHAPES[8:9] if "--only-product" in sys.argv else SHAPES
    prec = 1 if "--fp32" in sys.argv else 0
    for tile, rows, cols, K, batch, inplace, label in shapes:
        rc = lib.rgf_ktest_gemm_time(prec, tile, rows, cols, K, batch, inplace, 5, C.byref(ms))
        fl = 8.0 * rows * cols * K * batch
        print(f"| {label} | {ms.value * 1e3:.1f} | {fl / ms.value / 1e9:.1f} | rc={rc}", flush=True)
    if "--only-product" in sys.argv:
        return
    f, s = C.c_double(), C.c_double()
    for Mp in (512, 1024):
        rc = lib.rgf_ktest_lu_time(prec, Mp, Mp, 64, 3, C.byref(f), C.byref(s))
        print(f"LU Mp={Mp}, 64 energies: factor {f.value:.2f} ms, solves {s.value:.2f} ms rc={rc}", flush=True)


if __name__ == "__main__":
    main()
