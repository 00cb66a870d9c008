"""Write tests/golden/adjoint_gradient_64sq_20steps.txt: the oracle's
complex-step gradient of the integrated energy release with respect to the
20 rate parameters (lnA_r, E_r of the 10 reactions) on the adjoint workload
(7 species, smooth mode) at 64^2 zones over 20 steps.

    python tests/golden/make_adjoint_gradient.py [processes]

Calls only the oracle and the seeded input generator; one complex-step run
of the whole oracle per parameter, spread over worker processes.
"""
import multiprocessing as mp
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

SHAPE, NSTEPS = (64, 64), 20
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_gradient_64sq_20steps.txt")


def one(args):
    r, kind = args
    from threadpoolctl import threadpool_limits
    import sdc_inputs as si
    from oracle import adjoint, sdc
    w = si.workload("adjoint2d", shape=SHAPE)
    prob = sdc.Problem.from_workload(w)
    with threadpool_limits(limits=1):  # one thread per worker process
        g_lnA, g_E = adjoint.energy_gradient(w["U0"], w["dt"], NSTEPS, prob, which=kind, reactions=[r])
    return (g_lnA if kind == "lnA" else g_E)[0]


def main():
    import sdc_inputs as si
    w = si.workload("adjoint2d", shape=SHAPE)
    nr = w["network"]["nreact"]
    jobs = [(r, k) for k in ("lnA", "E") for r in range(nr)]
    procs = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()
    with mp.get_context("spawn").Pool(procs) as pool:
        g = pool.map(one, jobs, chunksize=1)
    with open(OUT, "w") as f:
        f.write("# Oracle complex-step gradient dJ_E/dtheta, adjoint workload (adjoint2d recipe: 7 species /\n"
                f"# 10 reactions, smooth mode) at {SHAPE[0]}x{SHAPE[1]} zones over {NSTEPS} steps with the\n"
                "# workload's dt.  J_E = dV sum_z sum_i q_i [rhoX_i(t0) - rhoX_i(tN)] (energy released).\n"
                "# Written by tests/golden/make_adjoint_gradient.py from oracle/ only.\n")
        f.write("dlnA: " + " ".join(repr(float(v)) for v in g[:nr]) + "\n")
        f.write("dE: " + " ".join(repr(float(v)) for v in g[nr:]) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
