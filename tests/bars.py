"""Per-channel parity bars of the arithmetic forms against the FP64 oracle.

A channel (or localized-SDFT bin) is held to its form's bar relative to its
own peak response, max |F_ref| over the pixels compared:
  - FP32 and the float16 hi/lo split (22 significant bits per operand): 1e-5;
  - the bfloat16 hi/lo split: 1e-3 (the matrix-core form's target);
  - single float16 products: 4e-3, single bfloat16 products: 4e-2 -- the
    worst errors measured over every tested configuration are 3.6e-3 and
    2.7e-2 (the localized SDFT of a one-row image under the mirror rule;
    1.3e-3 and 9.8e-3 on the 1024^2 metric bank), so these bars keep a
    margin of 1.1-1.5 and a channel 5 % wrong still fails.
Only where a channel's response nearly cancels (its peak below 1e-2 of
max |f|, e.g. a vertical channel of a three-row mirror-extended image whose
folded signal repeats every four rows) is the absolute rounding bound of
the form used instead: 8 u max|f| (|F| <= max|f| because the taps'
magnitudes sum to one; four operand roundings over two passes; u = 2^-9,
2^-12 for single bfloat16, float16 products, 2^-16, 2^-22 for their hi/lo
splits, 16 x 2^-24 for FP32 with its accumulation).  The count of such
channels is returned so that the tests can print it."""
import numpy as np

TOLS = {"fp32": 1e-5, "fp16_split": 1e-5, "bf16_split": 1e-3, "fp16": 4e-3, "bf16": 4e-2}
UNIT = {"fp32": 16 * 2.0 ** -24, "fp16_split": 2.0 ** -22, "bf16_split": 2.0 ** -16,
        "fp16": 2.0 ** -12, "bf16": 2.0 ** -9}
CANCEL = 1e-2


def channel_bars(prec, fmax, peak):
    """Absolute error bar per channel (array like peak) and the number of
    nearly cancelling channels that take the absolute rounding bound."""
    peak = np.asarray(peak, dtype=np.float64)
    cancel = peak < CANCEL * fmax
    bar = np.where(cancel, 8 * UNIT[prec] * fmax, TOLS[prec] * peak)
    return bar, int(cancel.sum())
