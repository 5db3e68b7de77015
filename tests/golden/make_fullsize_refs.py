"""Oracle displacements of the full-size parity cases, written once on the CPU.

    python tests/golden/make_fullsize_refs.py [case ...]

Calls only the oracle (monolithic sparse direct FP64 solves) on the seeded
workloads; each result is stored as tests/golden/fullsize/<case>_<hash>.npy,
where <hash> identifies the mesh, loads and state it was computed from
(see fullsize_key), so a test never compares against a reference of another
input.  Cases:

  random_boxes_40      linear solve of the 40^3 cube in 5^3 uneven boxes
                       (box sizes up to 5616 DOFs)
  tube_step0           first Newton step of the 16x128x64 tube from rest at
                       load factor 1/40 (0.4 mmHg)
  tube_step1           the Newton step at U_1 = U_0 + STEP1_SCALE dU_0 (a
                       stressed, non-equilibrium state; the full first step
                       of the nearly incompressible wall overshoots into states
                       with inverted elements) for the same load factor
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
OUT = os.path.join(HERE, "fullsize")

TUBE_TAU = 1.0 / 40.0
STEP1_SCALE = 0.25


def fullsize_key(mesh, *extra):
    """Hash of every input array of the mesh and of the extra arrays/scalars."""
    h = hashlib.sha256()
    for a in (mesh.xyz, mesh.hex8, mesh.elem_sub, mesh.mat, mesh.elem_mat, mesh.dir_dof, mesh.dir_val,
              mesh.body_force, mesh.fibers, mesh.pface, np.array([mesh.pressure])) + tuple(extra):
        if a is None:
            h.update(b"none")
        else:
            a = np.ascontiguousarray(np.asarray(a))
            h.update(str(a.dtype).encode() + str(a.shape).encode())
            h.update(a.tobytes())
    return h.hexdigest()[:16]


def path_for(case, key):
    return os.path.join(OUT, f"{case}_{key}.npy")


def case_random_boxes_40():
    from workloads import config_mesh
    from oracle import monolithic
    m = config_mesh("random_boxes_40")
    return [("random_boxes_40", fullsize_key(m), lambda: monolithic.solve_linear(m))]


def case_tube():
    from workloads import config_mesh
    from oracle import monolithic
    m = config_mesh("tube_16x128x64")
    U0 = np.zeros(m.n_dofs)
    out = []
    t0 = time.time()
    dU0, _ = monolithic.newton_increment(m, U0, TUBE_TAU)
    print(f"tube step 0: {time.time() - t0:.0f} s", flush=True)
    np.save(path_for("tube_step0", fullsize_key(m, U0, np.array([TUBE_TAU]))), dU0)
    out.append(("tube_step0", fullsize_key(m, U0, np.array([TUBE_TAU])), lambda: dU0))
    U1 = U0 + STEP1_SCALE * dU0
    t0 = time.time()
    dU1, _ = monolithic.newton_increment(m, U1, TUBE_TAU)
    print(f"tube step 1: {time.time() - t0:.0f} s", flush=True)
    out.append(("tube_step1", fullsize_key(m, U1, np.array([TUBE_TAU])), lambda: dU1))
    return out


CASES = {"random_boxes_40": case_random_boxes_40, "tube": case_tube}


def main(names):
    os.makedirs(OUT, exist_ok=True)
    for name in names or list(CASES):
        for case, key, fn in CASES[name]():
            t0 = time.time()
            u = np.asarray(fn(), dtype=np.float64)
            np.save(path_for(case, key), u)
            print(f"{case}: {u.size} values, key {key}, {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
