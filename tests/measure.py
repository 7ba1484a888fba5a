"""Measured-error bookkeeping of the FP32 parity checks.

Every FP32 comparison with the oracle prints the error it measured next to its
bound ("[measured] name: error (bound ...)"), so a GPU run of the suite lists the
figures the bounds come from.  Each bound is at most about four times the largest
error measured for that check on an MI355X (over its parameter cases).
"""


def check(name: str, err: float, bound: float) -> None:
    print(f"[measured] {name}: {err:.3e} (bound {bound:.1e})", flush=True)
    assert err <= bound, f"{name}: error {err:.3e} above the bound {bound:.1e}"


def max_rel_energy(hist, ref, fields=("energy",), floor=0.0):
    """Largest |got - ref| / max(floor, |ref|) over the steps, states and fields of
    two observable histories ([step][state] dicts)."""
    worst = 0.0
    for s in range(len(ref)):
        for i in range(len(ref[s])):
            for f in fields:
                g, r = hist[s][i][f], ref[s][i][f]
                worst = max(worst, abs(g - r) / max(floor, abs(r)))
    return worst
