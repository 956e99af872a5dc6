"""Write the stored oracle values used by the GPU tests.

Calls only the CPU oracle (and the seeded workload generator).  Run from the
repository root:  python tests/golden/make_golden.py
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def three_mode():
    """3 Kerr modes, cutoff 12, bitstring projector, T = 10 us, dt = 0.1 ns."""
    w = synth.three_mode_c1()
    t0 = time.time()
    out = oracle.evolve(w.system, oracle.product_sectors(w.factors), w.t_total, w.dt)
    vals = [oracle.expectation(w.system.cutoff, out, st) for st in w.states]
    return {"workload": w.name, "seed": 1, "t_total": w.t_total, "dt": w.dt,
            "states": [[k, [complex(x).real for x in v] if k == "fock" else
                        [[complex(x).real, complex(x).imag] for x in v]] for k, v in w.states],
            "values": [[v.real, v.imag] for v in vals], "oracle_seconds": time.time() - t0}


if __name__ == "__main__":
    data = three_mode()
    with open(os.path.join(HERE, "three_mode.json"), "w") as fh:
        json.dump(data, fh, indent=1)
    print(json.dumps(data)[:400])
