"""FP64 CPU oracle of the hybrid FNO-LBM hot path -- TEST INFRASTRUCTURE ONLY.

Only tests/, the package smoke check and the benchmark's CPU-baseline leg import
this package.  The GPU product path (paper_2604_27158_amd) never imports, links or
calls it, and it shares no code with that path: the lattice oracle is plain C
(lbm_oracle.c, FP64) and the FNO oracle plain numpy (fno.py, FP64, with an optional
BF16 operand-rounding mode).  Inputs come from paper_2604_27158_amd.workloads, which
holds no arithmetic of the method.
"""
