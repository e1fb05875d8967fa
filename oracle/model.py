"""Execution model of Section 4 (test infrastructure only; see package header).

Symbols follow Table 2: ``N`` = N_process (SPMD processes sharing one GPU),
``t_init`` = T_init, ``t_ctx`` = T_ctx_switch, ``t_in`` = T_data_in,
``t_comp`` = T_comp, ``t_out`` = T_data_out.  Every function is a closed
form printed in Section 4.1 / 4.2.3, written out as printed.

Readings taken where the text is silent or inconsistent:

* Classification (Section 4.2.3) defines compute-intensive (C-I) as
  ``t_in <= t_comp and t_out <= t_comp`` and I/O-intensive (IO-I) as
  ``t_in > t_comp and t_out > t_comp``.  The mixed case is not defined; it is
  classified "INT" (the paper's "Intermediate" class of the MM benchmark,
  Table 3) and gets the programming style with the smaller modelled time.
* The text after Eq. 3 states ``Eq2 < Eq3`` for C-I kernels, but
  ``Eq2 - Eq3 = (N-1)(t_in + t_out - t_comp)``, which is negative only when
  ``t_in + t_out < t_comp``.  ``paper_ps_choice`` keeps the paper's rule
  (C-I -> PS-1, IO-I -> PS-2); ``best_ps_choice`` takes the argmin.
* Eq. 1 counts the ``N - 1`` context switches between consecutive
  processes, as printed.
"""

from __future__ import annotations

import math

__all__ = [
    "eq1_total_no_vt",
    "eq2_total_ci_ps1",
    "eq3_total_ci_ps2",
    "eq4_total_ioi_ps1",
    "eq5_total_ioi_ps2_out_lt_in",
    "eq6_total_ioi_ps2_out_ge_in",
    "eq7_total_ioi_ps2",
    "eq8_speedup_ci",
    "eq9_speedup_ioi",
    "eq10_speedup_max_ci",
    "eq11_speedup_max_ioi",
    "classify",
    "paper_ps_choice",
    "best_ps_choice",
    "modelled_total",
]


def _check(n, *ts):
    if int(n) != n or n < 1:
        raise ValueError("N_process must be a positive integer")
    for t in ts:
        if not (t >= 0.0) or math.isinf(t):
            raise ValueError("times must be finite and non-negative")


def eq1_total_no_vt(n, t_init, t_ctx, t_in, t_comp, t_out):
    """Eq. 1: processes run one after another, each paying initialisation and
    its own send / compute / retrieve, with a context switch between each
    pair of consecutive processes."""
    _check(n, t_init, t_ctx, t_in, t_comp, t_out)
    return n * (t_init + t_in + t_comp + t_out) + (n - 1) * t_ctx


def eq2_total_ci_ps1(n, t_in, t_comp, t_out):
    """Eq. 2: C-I kernels under PS-1 (all sends, then all kernels, then all
    retrieves): every transfer is serial, all kernels overlap."""
    _check(n, t_in, t_comp, t_out)
    return n * (t_in + t_out) + t_comp


def eq3_total_ci_ps2(n, t_in, t_comp, t_out):
    """Eq. 3: C-I kernels under PS-2 (send, kernel, retrieve per stream):
    kernels serialise behind the implicit synchronisation of the previous
    retrieve, transfers hide under them."""
    _check(n, t_in, t_comp, t_out)
    return t_in + n * t_comp + t_out


def eq4_total_ioi_ps1(n, t_in, t_comp, t_out):
    """Eq. 4: IO-I kernels under PS-1, the same expression as Eq. 2."""
    _check(n, t_in, t_comp, t_out)
    return n * (t_in + t_out) + t_comp


def eq5_total_ioi_ps2_out_lt_in(n, t_in, t_comp, t_out):
    """Eq. 5: IO-I under PS-2 when ``t_out < t_in``: the input transfers set
    the pace, one kernel and one retrieve trail the last send."""
    _check(n, t_in, t_comp, t_out)
    return n * t_in + t_comp + t_out


def eq6_total_ioi_ps2_out_ge_in(n, t_in, t_comp, t_out):
    """Eq. 6: IO-I under PS-2 when ``t_out >= t_in``: the retrieves set the
    pace after the first send and kernel."""
    _check(n, t_in, t_comp, t_out)
    return t_in + t_comp + n * t_out


def eq7_total_ioi_ps2(n, t_in, t_comp, t_out):
    """Eq. 7: Eq. 5 and Eq. 6 combined,
    ``N max(t_in, t_out) + t_comp + min(t_in, t_out)``."""
    _check(n, t_in, t_comp, t_out)
    return n * max(t_in, t_out) + t_comp + min(t_in, t_out)


def eq8_speedup_ci(n, t_init, t_ctx, t_in, t_comp, t_out):
    """Eq. 8: speedup of the virtualised C-I case, Eq. 1 over Eq. 2."""
    return eq1_total_no_vt(n, t_init, t_ctx, t_in, t_comp, t_out) / eq2_total_ci_ps1(
        n, t_in, t_comp, t_out
    )


def eq9_speedup_ioi(n, t_init, t_ctx, t_in, t_comp, t_out):
    """Eq. 9: speedup of the virtualised IO-I case, Eq. 1 over Eq. 7."""
    return eq1_total_no_vt(n, t_init, t_ctx, t_in, t_comp, t_out) / eq7_total_ioi_ps2(
        n, t_in, t_comp, t_out
    )


def eq10_speedup_max_ci(t_init, t_ctx, t_in, t_comp, t_out):
    """Eq. 10: limit of Eq. 8 as N grows without bound,
    ``(t_init + t_in + t_comp + t_out + t_ctx) / (t_in + t_out)``."""
    _check(1, t_init, t_ctx, t_in, t_comp, t_out)
    return (t_init + t_in + t_comp + t_out + t_ctx) / (t_in + t_out)


def eq11_speedup_max_ioi(t_init, t_ctx, t_in, t_comp, t_out):
    """Eq. 11: limit of Eq. 9 as N grows without bound,
    ``(t_init + t_in + t_comp + t_out + t_ctx) / max(t_in, t_out)``."""
    _check(1, t_init, t_ctx, t_in, t_comp, t_out)
    return (t_init + t_in + t_comp + t_out + t_ctx) / max(t_in, t_out)


def classify(t_in, t_comp, t_out):
    """Kernel class of Section 4.2.3: "CI", "IOI", or "INT" for the mixed case
    the text leaves undefined."""
    if t_in <= t_comp and t_out <= t_comp:
        return "CI"
    if t_in > t_comp and t_out > t_comp:
        return "IOI"
    return "INT"


def paper_ps_choice(t_in, t_comp, t_out, n=2):
    """Programming style the paper assigns (end of Section 4.2.3 and
    Section 5): PS-1 for C-I kernels, PS-2 for IO-I kernels; the mixed class
    takes the style with the smaller modelled time for ``n`` processes."""
    cls = classify(t_in, t_comp, t_out)
    if cls == "CI":
        return "PS1"
    if cls == "IOI":
        return "PS2"
    return best_ps_choice(n, t_in, t_comp, t_out)


def modelled_total(style, n, t_in, t_comp, t_out):
    """Total GPU time of ``n`` virtualised processes under ``style``.

    PS-1 is Eq. 2 (= Eq. 4) for every class.  PS-2 is Eq. 3 when the kernel
    is C-I and Eq. 7 when it is IO-I; for the mixed class, which neither
    derivation covers, the larger of the two PS-2 expressions (in the C-I
    case Eq. 3 >= Eq. 7 and in the IO-I case Eq. 7 > Eq. 3, so the larger
    one is also the printed one there)."""
    if style == "PS1":
        return eq2_total_ci_ps1(n, t_in, t_comp, t_out)
    if style != "PS2":
        raise ValueError("style must be 'PS1' or 'PS2'")
    cls = classify(t_in, t_comp, t_out)
    if cls == "CI":
        return eq3_total_ci_ps2(n, t_in, t_comp, t_out)
    if cls == "IOI":
        return eq7_total_ioi_ps2(n, t_in, t_comp, t_out)
    return max(eq3_total_ci_ps2(n, t_in, t_comp, t_out), eq7_total_ioi_ps2(n, t_in, t_comp, t_out))


def best_ps_choice(n, t_in, t_comp, t_out):
    """Style with the smaller modelled total for ``n`` processes (ties go to
    the paper's choice for the class, PS-1 for the mixed class)."""
    p1 = modelled_total("PS1", n, t_in, t_comp, t_out)
    p2 = modelled_total("PS2", n, t_in, t_comp, t_out)
    if p1 < p2:
        return "PS1"
    if p2 < p1:
        return "PS2"
    return "PS2" if classify(t_in, t_comp, t_out) == "IOI" else "PS1"
