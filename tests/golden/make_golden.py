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


def quadratures():
    """4 Kerr modes, cutoff 8, product of quadratures prod_j (a_j + a_j^+)
    (16 off-diagonal sectors with Kerr phases of ~1.5e3 rad/us), T = 0.02 us:
    classical RK4 at dt = 1e-6 us, and the integrating-factor RK4 at dt = 1e-5
    us as a cross-check."""
    w = synth.grad_c3b()
    ops = oracle.product_sectors(w.factors)
    t0 = time.time()
    rk = oracle.expectation(w.system.cutoff, oracle.evolve(w.system, ops, w.t_total, w.dt), w.states[0])
    t_rk = time.time() - t0
    lw = oracle.expectation(w.system.cutoff, oracle.evolve_lawson(w.system, ops, w.t_total, 1e-5), w.states[0])
    return {"workload": w.name, "seed": 3, "t_total": w.t_total, "dt": w.dt,
            "state": [[complex(x).real, complex(x).imag] for x in w.states[0][1]],
            "value": [rk.real, rk.imag], "lawson_dt_1e-5": [lw.real, lw.imag],
            "rel_diff": abs(rk - lw) / abs(rk), "oracle_seconds": t_rk}


WRITERS = {"three_mode": three_mode, "quadratures": quadratures}

if __name__ == "__main__":
    for name in sys.argv[1:] or WRITERS:
        data = WRITERS[name]()
        with open(os.path.join(HERE, f"{name}.json"), "w") as fh:
            json.dump(data, fh, indent=1)
        print(name, json.dumps(data)[:300])
