"""Rounding-error model of the mixed (FP32 grid) IBDL operator, used as the
parity bar of mixed applies.

In the FP32 pipeline every stage rounds its results to FP32 (unit roundoff
u = 2^-24): the spread sums FP32-rounded weights and strengths, each FFT stage
and the symbol factor round the spectrum.  These errors spread over all
frequencies like white noise, while the exact spectrum of the dipole forcing
f = S~ q sits at high frequencies, where |lambda| is large.  L^-1 divides the
noise at every frequency by its own lambda, so the error field of u = L^-1 f
has root-mean-square size about

    u * sqrt(log2 n^d) * rms(f) * sqrt(mean_m 1/lambda_m^2)

(sqrt(log2 n^d) for the independent roundings of the log2 n^d FFT stages a
value passes through), and the interpolation, a weighted average whose weights
sum to 1, carries it to each of the M points.  The relative error of A q is
therefore about

    E = u * sqrt(log2 n^d) * rms(f) * sqrt(mean_m 1/lambda_m^2) * sqrt(M) / ||A q||_2.

Measured on MI355X over 2-D n = 256..1536 and 3-D n = 64..256 (alpha 1..1000,
both boundary conditions, 30 densities) the ratio of the measured error to E
lies between 0.26 and 1.49, over errors from 5e-9 to 3.5e-6; the bar is
MODEL_FACTOR * E.
"""
import math

import numpy as np

from oracle import ibdl_oracle as O

U32 = 2.0 ** -24
MODEL_FACTOR = 4.0


def mixed_model(st, q, aq):
    """E for density q on the oracle setup st, with aq = A q from the oracle."""
    f = O.spread_dipole(st, q)
    lam = O.symbol(st)
    nz = lam != 0.0
    inv2 = np.where(nz, 1.0 / np.where(nz, lam, 1.0), 0.0) ** 2
    rms_f = float(np.sqrt(np.mean(f * f)))
    return (U32 * math.sqrt(math.log2(st.n ** st.dim)) * rms_f * math.sqrt(float(np.mean(inv2))) *
            math.sqrt(st.m) / float(np.linalg.norm(aq)))
