"""Shared comparison helpers for the GPU parity tests (not a test module)."""
import numpy as np


def field_errors(z, zo, field_of_row):
    """Relative 2-norm difference of z against zo within each field."""
    out = []
    for f in range(int(field_of_row.max()) + 1):
        m = field_of_row == f
        den = np.linalg.norm(zo[m])
        out.append(np.linalg.norm(z[m] - zo[m]) / den if den > 0 else np.linalg.norm(z[m]))
    return out


def assert_fields_close(z, zo, field_of_row, tol, tag=""):
    """Per-field bound: one field's norm must not hide another's error (the
    fields' parts of M^-1 r differ by orders of magnitude)."""
    err = field_errors(z, zo, field_of_row)
    assert max(err) <= tol, (tag, [f"{e:.2e}" for e in err])
    return err
