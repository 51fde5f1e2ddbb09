"""FP64 CPU oracle of the fluctuating two-component LBM + particle step.

Test infrastructure only: imported by tests/, the smoke check and the
CPU-baseline leg of the benchmark, never by the HIP package.
"""
