"""Write flops_per_unit.json: algorithmic flops of the CT-MHD step per unit of
work, measured with the oracle's counting scalar type (add/sub, mul, div and
sqrt each count as one flop; comparisons are not counted).

The oracle is deliberately naive (it reconstructs each interface from both
sides and re-derives two-step edge reconstructions per corner), so its raw
totals are not algorithmic.  The counter tags every 1D reconstruction
separately; the table below charges each reconstruction once per cell and
direction, which is what the method needs:
  face    : Riemann solve, flux, alpha, u* per face  + 7 reconstructions
  edge    : corner EMFs + LD04 (+ eta j) per edge    + edge reconstructions
            (Q26: 4, B25a: 6, FS18: 12 per edge)
  cell    : primitives, update, dt per cell update
Run: python tests/golden/make_flops.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2609_10816_amd import inputs  # noqa: E402

EDGE_RECON = {"q26": 4, "b25a": 6, "fs18": 12}


def flops(c, ph):
    return sum(v for k, v in c[ph].items() if k != "cmp")


def main():
    n = 16
    cons, bf, info = inputs.turbulent_box((n, n, n), mach=5.0, b0=(0.1, 0.0, 0.0),
                                          db_rms=0.05, seed_v=1, seed_a=2)
    N = n ** 3
    table = {"source": "oracle counting type on the 16^3 Mach-5 turbulent box, FOFC off "
                       "(no cell flagged), one step; per-unit figures",
             "entries": {}}
    for recon in ["pc", "plm", "ppm"]:
        for emf in ["q26", "b25a", "fs18"]:
            for eta in [0.0, 1e-3]:
                c = oracle.count_step(dict(recon=recon, emf=emf, eta=eta, fofc=False), cons, bf,
                                      info["dx"])
                per_recon = flops(c, "recon") / max(c["recon_calls"], 1)
                face = flops(c, "face") / (6 * N) + 7 * per_recon
                edge = flops(c, "emf") / (6 * N) + EDGE_RECON[emf] * per_recon
                cell = (flops(c, "update") + flops(c, "dt") + flops(c, "prim")) / N
                key = f"{recon}/{emf}/eta{'>0' if eta > 0 else '=0'}"
                table["entries"][key] = {
                    "recon_flops": per_recon,
                    "face_flops": face,
                    "edge_flops": edge,
                    "cell_flops": cell,
                    "cell_update_flops": 6 * face + 6 * edge + cell,
                }
    out = os.path.join(HERE, "flops_per_unit.json")
    with open(out, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print(out)


if __name__ == "__main__":
    main()
