"""Test-side glue: run the GPU path and the oracle on the same seeded
instances and compare."""
import numpy as np

from tests.conftest import to_oracle


def as_dtype(inst, dtype):
    """The instance with its data rounded to the GPU run's precision, so that
    the oracle and the GPU solve the same problem."""
    if dtype != "f32":
        return inst
    out = dict(inst)
    for k in ("coeff", "rhs", "bc_values"):
        out[k] = np.asarray(inst[k], np.float32).astype(np.float64)
    return out


def gpu_solve(instances, dtype="f32", **opts):
    import torch
    from paper_2502_18377_amd.api import Problem, pack
    tdt = torch.float32 if dtype == "f32" else torch.float64
    pk = pack(instances, dtype=tdt, device="cuda")
    prob = Problem(pk["coeff"], pk["rhs"], pk["bc_values"], pk["shapes"], pk["steps"], pk["bc"], pk["mset"], **opts)
    z, info = prob.solve()
    torch.cuda.synchronize()
    zs = [t.double().cpu().numpy() for t in prob.split(z)]
    return prob, zs, info


def oracle_solve(inst):
    from oracle.system import assemble
    from oracle.solve import solve_kkt
    A, d, rows = assemble(to_oracle(inst))
    z, lam, lu = solve_kkt(A, d)
    V = 1 + 2 * len(inst["shape"])
    return z.reshape((V,) + tuple(inst["shape"])), (A, d, rows, z, lam, lu)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def normal_relres(inst, zgpu):
    from oracle.system import assemble
    from oracle.solve import normal_residual
    A, d, _ = assemble(to_oracle(inst))
    return normal_residual(A, d, zgpu.reshape(-1))
