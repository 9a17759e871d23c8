"""Expected outputs of the 256-patch coefficient-aware batch at sampled entries, from the oracle only.

The batch: 256 3D Taylor-Hood patches, n_el per direction uniform in [8, 48],
p uniform in {2..5} (seed 3), the sine map G(eta)_j = eta_j + 0.1 sin(pi eta_j)
with viscosity 1 + 0.5 sin(2 pi x_1) cos(2 pi x_2), one Gaussian residual per
patch drawn after the descriptors; each patch's block vector is z = P_D^{-1} r
with the coefficient-aware blocks of Sec. 6 and the Appendix.

The oracle's setup of the largest patches takes minutes each, so the values a
GPU run compares against are computed here once: for the 8 largest patches
and 8 further patches drawn with a fixed seed, every block of z at the entries
of a few whole pencils per direction (the two corner pencils, which sit in the
first and the last (ragged) tiles of every pass, and two drawn pencils), with
each block's largest magnitude and RMS over all of its entries.

Only ``oracle/`` computes values here; ``paper_1712_00403_amd.workloads``
supplies the seeded patch descriptors and residual draws.

Usage: python tests/golden/make_batch_golden.py   (writes batch_256_sampled.npz beside this file)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "batch_256_sampled.npz")
COUNT, SEED = 256, 3
N_LARGEST, N_DRAWN, PICK_SEED = 8, 8, 7


def block_sizes(n_el, p):
    """Orders of the velocity and pressure spaces of a TH patch, from the oracle's assembly."""
    from oracle.assemble import pressure_1d, taylor_hood_velocity_1d
    nv = tuple(taylor_hood_velocity_1d(n, p)[1].shape[0] for n in n_el)
    nq = tuple(pressure_1d(n, p).shape[0] for n in n_el)
    return nv, nq


def patch_blocks(n_el, p):
    """Shapes of the blocks of a patch's block vector: d velocity blocks then the pressure block."""
    nv, nq = block_sizes(n_el, p)
    return [nv] * len(n_el) + [nq]


def selected(sizes):
    """Indices of the checked patches: the N_LARGEST largest block vectors, then N_DRAWN drawn from the rest."""
    order = sorted(range(len(sizes)), key=lambda i: (-sizes[i], i))
    big = order[:N_LARGEST]
    rest = sorted(order[N_LARGEST:])
    drawn = sorted(int(i) for i in np.random.default_rng(PICK_SEED).choice(rest, N_DRAWN, replace=False))
    return big + drawn


def pencil_entries(shape, key):
    """Flat indices (i_1 fastest) of the sampled pencils of a block of ``shape``.

    Per direction a: the pencils along a through the two corners of the cross
    section (all other indices 0, all other indices last) and two cross-section
    positions drawn from default_rng(key + a).
    """
    shape = tuple(int(s) for s in shape)
    d = len(shape)
    strides = [int(np.prod(shape[:j])) for j in range(d)]
    idx = []
    for a in range(d):
        others = [j for j in range(d) if j != a]
        rng = np.random.default_rng(key + a)
        crosses = [[0] * len(others), [shape[j] - 1 for j in others]]
        crosses += [[int(rng.integers(0, shape[j])) for j in others] for _ in range(2)]
        for c in crosses:
            base = sum(ci * strides[j] for ci, j in zip(c, others))
            idx.append(base + strides[a] * np.arange(shape[a]))
    return np.unique(np.concatenate(idx)).astype(np.int64)


def batch_inputs():
    """Patch descriptors, block-vector sizes and residuals of the batch, in draw order."""
    from paper_1712_00403_amd import workloads
    patches, rng = workloads.batch_patches(COUNT, seed=SEED)
    sizes = [int(sum(np.prod(s) for s in patch_blocks(n_el, p))) for n_el, p in patches]
    res = workloads.batch_residuals(rng, sizes)
    return patches, sizes, res


def main():
    from oracle.fd import FDFactors, block_apply
    from oracle.geometry import GeometryBlocks
    from paper_1712_00403_amd import workloads
    patches, sizes, res = batch_inputs()
    pick = selected(sizes)
    geo = workloads.sine_geometry(3)
    out = {"patches": np.array(pick, dtype=np.int64)}
    for i in pick:
        t0 = time.perf_counter()
        n_el, p = patches[i]
        gb = GeometryBlocks(n_el, p, geo)
        facs = [FDFactors(gb.vel_K[k], gb.vel_M[k]) for k in range(3)]
        zo = block_apply(facs, gb.pres_M, res[i], pres_scale=gb.pres_scale, vel_scales=gb.vel_scales)
        off = 0
        for b, shape in enumerate(patch_blocks(n_el, p)):
            nb = int(np.prod(shape))
            zb = zo[off:off + nb]
            idx = pencil_entries(shape, 1000 * i + 10 * b)
            out[f"p{i}_b{b}_idx"] = idx
            out[f"p{i}_b{b}_val"] = zb[idx]
            out[f"p{i}_b{b}_max"] = np.array(np.max(np.abs(zb)))
            out[f"p{i}_b{b}_rms"] = np.array(np.sqrt(np.mean(zb * zb)))
            off += nb
        assert off == sizes[i]
        print(f"patch {i} n_el={n_el} p={p}: {time.perf_counter() - t0:.1f} s", flush=True)
        del gb, facs, zo
    np.savez_compressed(OUT, **out)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
