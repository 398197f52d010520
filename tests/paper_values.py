"""Readers of the paper's printed values stored under tests/golden/ (each
file names the table or passage it copies)."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line.split()


def table1():
    """Table 1 (Sec. 2.5) by shape: {"sup_tau", "sup_xi", "kstar_A",
    "tested": [(k, converges), ...], "errors": [...]}."""
    out = {}
    for shape, sup_tau, sup_xi, ks, k, err, result in _rows("table1_annulus.txt"):
        d = out.setdefault(int(shape), {"sup_tau": float(sup_tau), "sup_xi": float(sup_xi),
                                        "kstar_A": float(ks), "tested": [], "errors": []})
        d["tested"].append((float(k), result == "converges"))
        d["errors"].append(float(err))
    return out


def fig2_crossings():
    """{grid spacing: k above which rho(G) > 1} stated with the Sec. 2.4 figure."""
    return {float(h): float(k) for h, k in _rows("fig2_spectral_radius.txt")}
