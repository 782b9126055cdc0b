"""Algorithmic operation counts of the GPU kernels (FP64 flops: add, multiply,
divide and square root count 1, a fused multiply-add counts 2).

They count the arithmetic each kernel's formulation needs, not the
instructions it issues: lane reductions, padding and index arithmetic are
left out.  Per neighbor entry (one (i, j) pair of the CSR) and per particle:

k_moments        per pair: displacement, weight and xi (15) + the 84 weighted
                 monomials of degree <= 6 built from shared partial products
                 (32 multiplies, 28 adds, 56 fused multiply-adds)        = 187
k_factor<3>      per particle: equilibration (20 sqrt, 20 div, 420 mul),
                 20x20 Cholesky (20 sqrt, 20 div, 190 mul, 1330 FMA),
                 three unit-vector solves (2234), output scaling (120)   = 5704
k_apply_rhs      per pair: geometry and weight (15), basis (16), three
                 operator rows G p (60 FMA), w (3), field differences (7),
                 gradient accumulation (21 FMA)                          = 203
                 per particle: gradient scaling (21) + right-hand side (45) = 66
k_adj_pairs      per pair: geometry and dw/dq (18), basis (16),
                 G p and K p (120 FMA), h (7 sub, 21 FMA), dfbar (42),
                 wbar (5), pbar = w (G^T b - K^T a) (120 FMA, 20 mul),
                 basis gradient (25), xibar over the 30 nonzero basis
                 derivatives (30 FMA), dbar (12), sums (10)               = 683
k_adj_gather     memory bound: 80 B per pair record, 232 B per particle.

FP64 data form (the fit coefficients are solved for, and taped with the
operator rows for the reverse mode):
k_fit_b<7>       per pair: geometry and weight (15), basis (16), per field
                 w df (2) and 20 FMA (40), seven fields                   = 325
k_moments_factor_fit<3>  per pair: the moments as k_moments            = 187
                 per particle: equilibration + Cholesky (3330), three
                 unit-vector solves (2234), seven general solves (7 x 820),
                 row norms of the screen (120), output scaling (260)      = 11684
k_rows_rhs_finish per particle: gradient scaling (21) + right-hand side   = 66
k_adj_u          per particle: pointwise adjoint                          = 150
k_adj_pairs_w    as k_adj_pairs; the owner's K = Ubar C^T (840 per
k_adj_pairs_p    particle) and the tile schedule's LDS sums (adds that
k_adj_pairs_t    replace a record's write and the gather's adds) are left
                 out of the count.

Mixed form without a tape (FP32 arithmetic after the FP64 displacement,
FP64 factor and solves; counted the same way, whatever the precision; a
mixed call with a tape runs the FP64 data form above):
k_moments<fp32>  as k_moments                                            = 187
k_mixed_b        per pair: geometry and weight (15), basis (16), per field
                 w df (2) and 20 FMA (40), seven fields                   = 325
k_mixed_factor   per particle: equilibration + Cholesky (3330), seven
                 general solves (7 x 820), three unit-vector solves (2234),
                 inverse-norm estimate (two solves 1640, norms 80),
                 output scaling (200)                                     = 13224
k_mixed_resid    per pair: geometry (15), basis (16), per field the FP32
                 fit (40), residual (3) and dB update (40), seven fields  = 612
                 per particle: E C + G dB (7 x 3 x 20 FMA + 21)           = 861
k_mixed_rhs_finish per particle: gradient scaling (21) + right-hand side  = 66

Operator-level refinement (the mixed form's default for three rows):
k_mixed_screen   per particle: equilibration + Cholesky (3330), three
                 unit-vector solves (2234), inverse-norm estimate (1720),
                 output scaling (120)                                     = 7404
k_mixed_gta      per pair and pass of three rows: geometry and weight (15),
                 basis (16), G~ p (60 FMA), w G~ p (3), M update (60 FMA) = 274
k_mixed_refine   per particle and three rows: equilibration + Cholesky
                 (3330), scaling in (60), three general solves (2460),
                 2 G~ - S x (60 mul, 60 FMA)                              = 6030
k_apply_rhs<fp32> as k_apply_rhs (FP64 operator weights, FP32 sums)       = 203
                 per particle                                             = 66
"""

PER_PAIR = {
    "k_moments": 187,
    "k_moments<fp32>": 187,
    "k_mixed_b": 325,
    "k_fit_b<7>": 325,
    "k_mixed_resid": 612,
    "k_apply_rhs": 203,
    "k_apply_rhs<fp32>": 203,
    "k_mixed_gta": 274,
    "k_adj_pairs": 683,
    "k_adj_pairs_w": 683,
    "k_adj_pairs_p": 683,
    "k_adj_pairs_t": 683,
    "k_moments_factor_fit<3>": 187,
}
PER_PARTICLE = {
    "k_factor<3>": 5704,
    "k_moments_factor_fit<3>": 11684,
    "k_rows_rhs_finish": 66,
    "k_adj_u": 150,
    "k_mixed_factor": 13224,
    "k_mixed_resid": 861,
    "k_mixed_rhs_finish": 66,
    "k_apply_rhs": 66,
    "k_apply_rhs<fp32>": 66,
    "k_mixed_screen": 7404,
    "k_mixed_refine": 6030,
}
BYTES_PER_PAIR = {"k_adj_gather": 80}
BYTES_PER_PARTICLE = {"k_adj_gather": 232}


def flops(kernel: str, n: int, nnz: int) -> float:
    return PER_PAIR.get(kernel, 0) * nnz + PER_PARTICLE.get(kernel, 0) * n


def bytes_moved(kernel: str, n: int, nnz: int) -> float:
    return BYTES_PER_PAIR.get(kernel, 0) * nnz + BYTES_PER_PARTICLE.get(kernel, 0) * n


# MI355X peaks: FP64 vector = 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz.
PEAK_FP64_VALU = 256 * 4 * 16 * 2 * 2.4e9  # 78.6 TFLOP/s
PEAK_HBM = 8.0e12
