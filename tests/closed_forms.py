"""Closed-form effective properties used to pin the oracle.

These are textbook results independent of the Lippmann--Schwinger
discretisation: exact laminate homogenisation (layers normal to e1) and the
Hashin--Shtrikman bounds.  They are written here, away from ``oracle/``, so
that a mistake in the oracle cannot also hide in its check.
"""
import math

import numpy as np


def scalar_laminate(fractions, conductivities):
    """Layers of isotropic conductivities normal to e1: (harmonic, arithmetic)."""
    f = np.asarray(fractions, dtype=float)
    a = np.asarray(conductivities, dtype=float)
    return 1.0 / np.sum(f / a), float(np.sum(f * a))


# Mandel indices: traction-like components (11, 13, 12) and in-plane ones
# (22, 33, 23) for a laminate with normal e1.
_T = [0, 4, 5]
_I = [1, 2, 3]


def elastic_laminate(fractions, stiffnesses):
    """Exact effective 6x6 Mandel stiffness of a laminate with normal e1.

    In every layer the in-plane strains (22, 33, 23) equal the macroscopic
    ones and the tractions (11, 12, 13) are uniform; eliminating the
    traction-direction strains layer by layer and averaging gives the
    effective tensor (the classical partial-inversion average)."""
    f = np.asarray(fractions, dtype=float)
    Cs = [np.asarray(C, dtype=float) for C in stiffnesses]
    inv_tt = sum(fi * np.linalg.inv(C[np.ix_(_T, _T)]) for fi, C in zip(f, Cs))
    inv_tt_ti = sum(fi * np.linalg.inv(C[np.ix_(_T, _T)]) @ C[np.ix_(_T, _I)] for fi, C in zip(f, Cs))
    it_inv = sum(fi * C[np.ix_(_I, _T)] @ np.linalg.inv(C[np.ix_(_T, _T)]) for fi, C in zip(f, Cs))
    schur = sum(fi * (C[np.ix_(_I, _I)] - C[np.ix_(_I, _T)] @ np.linalg.inv(C[np.ix_(_T, _T)]) @ C[np.ix_(_T, _I)])
                for fi, C in zip(f, Cs))
    Ctt = np.linalg.inv(inv_tt)
    Cti = Ctt @ inv_tt_ti
    Cit = it_inv @ Ctt
    Cii = schur + it_inv @ Cti
    out = np.zeros((6, 6))
    out[np.ix_(_T, _T)] = Ctt
    out[np.ix_(_T, _I)] = Cti
    out[np.ix_(_I, _T)] = Cit
    out[np.ix_(_I, _I)] = Cii
    return out


def hashin_shtrikman_scalar(f_incl, a_incl, a_mat, d):
    """HS bounds on the isotropic effective conductivity of a two-phase
    statistically isotropic composite in d dimensions."""
    lo_base, hi_base = (a_mat, a_incl) if a_mat < a_incl else (a_incl, a_mat)
    f_lo = f_incl if a_mat < a_incl else 1.0 - f_incl
    a_lo_other = a_incl if a_mat < a_incl else a_mat
    lower = lo_base + f_lo / (1.0 / (a_lo_other - lo_base) + (1.0 - f_lo) / (d * lo_base))
    f_hi = 1.0 - f_lo
    upper = hi_base + f_hi / (1.0 / (lo_base - hi_base) + (1.0 - f_hi) / (d * hi_base))
    return lower, upper


def keller_dykhne(a1, a2):
    """Effective conductivity of the 2D checkerboard: sqrt(a1 a2)."""
    return math.sqrt(a1 * a2)
