"""Block-diagonal Stokes preconditioner P_D = diag(P_V,1, .., P_V,d, P_Q) on the device.

P_D of eq. P_D (Sec. 4) with the simple blocks of Sec. 5 (eq. prec3D_TH,
eq. precQ): each velocity block is a Kronecker sum applied by FD, the pressure
block a Kronecker product of mass matrices applied by FD with Lambda = I. The
univariate factors come from the library's own assembly (fd_assemble_1d); the
apply of all blocks of all residuals is one fd_apply_batched call.

Block vectors are [u_1; ..; u_d; p] with the velocity components first, as in
the Stokes matrix of Sec. 3; a batch of residuals is residual-major.
"""
import numpy as np

from . import fd


def block_factors(spec):
    """(Ks, Ms) of one block from the library's assembly (Ks None for mass-only; Nitsche factors where named)."""
    Ks, Ms = [], []
    for f in spec.dirs:
        K, M = fd.assemble_1d(f.n_el, f.degree, f.regularity, f.dirichlet)
        if f.nitsche > 0:  # the RT blocks' Nitsche-modified stiffness
            K = fd.nitsche_stiffness_1d(f.n_el, f.degree, f.regularity, f.nitsche)
        Ks.append(K)
        Ms.append(M)
    return (None if spec.mass_only else Ks), Ms


class BlockPreconditioner:
    """Plans for every block of a workloads.Problem.

    ``factors`` / ``weights`` / ``diag_targets`` (one entry per block) replace
    the simple blocks' factors, direction weights and (absent) diagonal
    scalings, e.g. with those of the coefficient-aware blocks (``geometry``).
    """

    def __init__(self, problem, precision="f64", diag_targets=None, factors=None, weights=None,
                 pressure="fd"):
        """``pressure``: "fd" applies the unscaled mass-only block by FD with Lambda = I,
        "banded" by banded Cholesky solves per mode (the O(p n_Q) route of Sec. 5.2)."""
        if pressure not in ("fd", "banded"):
            raise ValueError("pressure route must be 'fd' or 'banded'")
        self.problem = problem
        self.precision = precision
        self.plans = []
        self.sizes = []
        try:
            for bi, spec in enumerate(problem.blocks):
                Ks, Ms = factors[bi] if factors is not None else block_factors(spec)
                dt = None if diag_targets is None else diag_targets[bi]
                w = np.asarray(spec.weights if weights is None else weights[bi], dtype=np.float64)
                banded = pressure == "banded" and Ks is None and dt is None
                plan = fd.Plan(Ks, Ms, weights=None if banded else w, diag_target=dt, precision=precision,
                               banded=banded)
                self.plans.append(plan)
                self.sizes.append(plan.N)
        except BaseException:
            # a block that fails (a device-memory cap, an exhausted device)
            # releases the plans of the blocks before it at once
            self.close()
            raise
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        self.N = int(self.offsets[-1])
        self.io_dtype = self.plans[0].io_dtype

    def works(self, r_ptr, z_ptr, nrhs, ld=None, elem_bytes=None):
        ld = self.N if ld is None else ld
        eb = elem_bytes or (8 if self.io_dtype == "float64" else 4)
        return [(p, r_ptr + int(o) * eb, z_ptr + int(o) * eb, nrhs, ld)
                for p, o in zip(self.plans, self.offsets[:-1])]

    def apply(self, r, z=None, stream=None):
        """z = P_D^{-1} r for a torch device tensor of shape (nrhs, N_block) or (N_block,)."""
        import torch
        dev = self.plans[0].device
        if z is None:
            fd.check_vectors(r, None, self.N, self.io_dtype, dev, exact=True)
            z = torch.empty_like(r)
        fd.check_vectors(r, z, self.N, self.io_dtype, dev, exact=True)
        r2 = r.reshape(-1, r.shape[-1])
        fd.apply_batched(self.works(r.data_ptr(), z.data_ptr(), r2.shape[0]), stream)
        return z

    def graph(self, r, z, warmup=2):
        """A HIP graph of z = P_D^{-1} r on these two buffers; ``.replay()`` reruns it.

        The launches of one apply are recorded once (on a side stream, after
        ``warmup`` eager applies there), so a replay is one submission instead
        of one per kernel: for small blocks the apply is launch-bound. The
        apply records no memset or host synchronization, so its replays are
        exact; r's contents may change between replays, its address may not.
        """
        import torch
        dev = self.plans[0].device
        fd.check_vectors(r, z, self.N, self.io_dtype, dev, exact=True)
        side = torch.cuda.Stream(device=r.device)
        side.wait_stream(torch.cuda.current_stream(r.device))
        with torch.cuda.stream(side):
            for _ in range(warmup):
                self.apply(r, z, stream=side)
        torch.cuda.current_stream(r.device).wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            self.apply(r, z, stream=side)
        return g

    def close(self):
        for p in self.plans:
            p.close()
