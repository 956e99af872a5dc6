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


def quadratures(cutoff=8):
    """4 Kerr modes, cutoff 8, product of quadratures prod_j (a_j + a_j^+)
    (16 off-diagonal sectors with Kerr phases of ~1.5e3 rad/us), T = 0.02 us:
    classical RK4 at dt = 1e-6 us, and the integrating-factor RK4 at dt = 1e-5
    us as a cross-check."""
    w = synth.grad_c3b(cutoff=cutoff)
    ops = oracle.product_sectors(w.factors)
    t0 = time.time()
    rk = oracle.expectation(w.system.cutoff, oracle.evolve(w.system, ops, w.t_total, w.dt), w.states[0])
    t_rk = time.time() - t0
    lw = oracle.expectation(w.system.cutoff, oracle.evolve_lawson(w.system, ops, w.t_total, 1e-5), w.states[0])
    return {"workload": w.name, "cutoff": cutoff, "seed": 3, "t_total": w.t_total, "dt": w.dt,
            "state": [[complex(x).real, complex(x).imag] for x in w.states[0][1]],
            "value": [rk.real, rk.imag], "lawson_dt_1e-5": [lw.real, lw.imag],
            "rel_diff": abs(rk - lw) / abs(rk), "oracle_seconds": t_rk}


def _single_modes(system, factors, state, steps, dt, sens=False):
    """Per mode of a product observable on the diagonal sector: the oracle's
    single-mode expectation value (and its parameter sensitivities K, Delta,
    gamma1, gamma_phi).  The N-mode value is their product: there the
    generator is a sum of commuting single-mode generators."""
    vals, grads = [], []
    for j, nc in enumerate(system.cutoff):
        sj = synth.System((nc,), system.detuning[j:j + 1], system.kerr[j:j + 1], [[0.0]],
                          system.gamma1[j:j + 1], system.gamma_phi[j:j + 1], system.n_th[j:j + 1])
        ops = oracle.product_sectors([factors[j]])
        st = (state[0], [state[1][j]])
        if sens:
            fin, sp = oracle.evolve_sens(sj, ops, steps * dt, dt, nthreads=1)
            grads.append([oracle.expectation((nc,), s_, st) for s_ in sp])
        else:
            fin = oracle.evolve_steps(sj, ops, steps, dt, nthreads=1)
        vals.append(oracle.expectation((nc,), fin, st))
    return vals, grads


def _prod(xs):
    out = 1.0 + 0.0j
    for x in xs:
        out *= x
    return out


def workloads():
    """Full-horizon expectation values of the benchmark workloads, each a
    product of single-mode oracle runs (exact on the diagonal sector up to
    RK4's O(h^5) splitting term):
    * 10 Kerr modes, cutoff 6, parity-weighted projector, T = 2 us, dt = 0.05 ns;
    * the 96 batch members at T = 1 us, dt = 0.1 ns;
    * the 4-mode cutoff-16 gradient workload at T = 5 us, dt = 0.1 ns: J and
      dJ/dtheta in the library's parameter order (K[N], chi[i<j], Delta[N],
      gamma1[N], gamma_phi[N]); only the gamma1 entries differ from zero by
      more than the oracle's rounding."""
    t0 = time.time()
    w = synth.large_c4()
    vals, _ = _single_modes(w.system, w.factors, w.states[0], w.n_steps, w.dt)
    ten = {"workload": w.name, "seed": 4, "t_total": w.t_total, "dt": w.dt, "steps": w.n_steps,
           "value": [_prod(vals).real, _prod(vals).imag]}
    batch = []
    for b in synth.batch_c2():
        vals, _ = _single_modes(b.system, b.factors, b.states[0], b.n_steps, b.dt)
        batch.append({"name": b.name, "steps": b.n_steps, "value": [_prod(vals).real, _prod(vals).imag]})
    g = synth.grad_c3()
    n = g.system.n_modes
    vals, grads = _single_modes(g.system, g.factors, g.states[0], g.n_steps, g.dt, sens=True)
    J = _prod(vals)
    npair = n * (n - 1) // 2
    dJ = [0.0j] * (n + npair + 3 * n)  # chi: no single-mode counterpart; zero on the diagonal sector
    for j in range(n):
        rest = _prod([vals[i] for i in range(n) if i != j])
        for k, slot in enumerate((j, n + npair + j, n + npair + n + j, n + npair + 2 * n + j)):
            dJ[slot] = grads[j][k] * rest  # K_j, Delta_j, gamma1_j, gamma_phi_j
    grad = {"workload": g.name, "seed": 3, "t_total": g.t_total, "dt": g.dt, "steps": g.n_steps,
            "value": [J.real, J.imag], "grad": [[x.real, x.imag] for x in dJ]}
    return {"ten_mode": ten, "batch": batch, "gradient": grad, "oracle_seconds": time.time() - t0}


def small_gradient():
    """The gradient of a small off-diagonal workload (4 Kerr modes, cutoff 5,
    product of quadratures: 16 sectors of 4^4 points), T = 0.02 us at
    dt = 1e-5 us (2,000 steps): J and the oracle's forward sensitivities in
    the library's parameter order."""
    w = synth.grad_c3b(cutoff=5, t_total=0.02, dt=1e-5)
    t0 = time.time()
    fin, sens = oracle.evolve_sens(w.system, oracle.product_sectors(w.factors), w.t_total, w.dt)
    J = oracle.expectation(w.system.cutoff, fin, w.states[0])
    dJ = [oracle.expectation(w.system.cutoff, sp, w.states[0]) for sp in sens]
    return {"workload": w.name, "seed": 3, "t_total": w.t_total, "dt": w.dt, "steps": w.n_steps,
            "value": [J.real, J.imag], "grad": [[x.real, x.imag] for x in dJ], "oracle_seconds": time.time() - t0}


WRITERS = {"three_mode": three_mode, "quadratures": quadratures, "quadratures6": lambda: quadratures(6),
           "workloads": workloads, "small_gradient": small_gradient}

if __name__ == "__main__":
    for name in sys.argv[1:] or WRITERS:
        data = WRITERS[name]()
        with open(os.path.join(HERE, f"{name}.json"), "w") as fh:
            json.dump(data, fh, indent=1)
        print(name, json.dumps(data)[:300])
