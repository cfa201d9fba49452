"""Error margins of the GPU parity tests: every check can report its worst error as a
fraction of its bound.  With COSMO_MARGIN_LOG set to a file name, each report appends
one line "label<TAB>err<TAB>bound<TAB>err/bound" to it, so a run of the suite records
how close each bound is to being reached (nothing is written otherwise)."""
import os


def note(label, err, bound):
    path = os.environ.get("COSMO_MARGIN_LOG")
    if not path:
        return
    err = float(err)
    bound = float(bound)
    with open(path, "a") as f:
        f.write(f"{label}\t{err:.3e}\t{bound:.3e}\t{err / bound if bound else float('inf'):.3f}\n")
