"""Oracle computations run in spawned worker processes by the GPU tests (CPU only: this
module imports neither torch nor the library)."""
import psl_inputs as pi
from oracle import psl_oracle as O


def c3_reference(seed, tol=1e-12):
    """The oracle's x for the 256x256x128 channelized workload with this seed: its own
    assembly, connected-component labels and DEF1 solve to relative residual `tol`.
    Returns (x, iterations, relative residual, d)."""
    from threadpoolctl import threadpool_limits
    with threadpool_limits(2):
        p = pi.config("c3", seed=seed)
        A, b = O.assemble(p.K, p.grid, p.dirichlet_mask, p.q)
        lab, d = O.levelset_components(p.grid, p.K, p.nsub, p.thr)
        r = O.dpcg(A, b, O.deflation_matrix(lab, d), tol=tol)
        return r.x, r.iters, r.relres, d
