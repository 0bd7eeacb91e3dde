"""Seeded synthetic workloads of the approximate Kappa generator.

The only module shared by the tests' two sides (GPU library and CPU oracle)
and by the benchmark.  It holds sizes, seeds and input generators; none of
the sampler's arithmetic.  The paper uses no dataset: its inputs are just
(kappa, theta, N, seed), and these configurations are its workloads.

  C1  plain method: 1e6 particles, kappa 3, theta 1, FP64, seed 0, counter =
      particle index (the size of the paper's first test, Sec. 5).
  C2  single-species sweep: 1e8 particles for each kappa in {1.6, 2, 3, 4, 6,
      10}, theta 1, seed 1 (the paper's third test uses 1e8 particles and
      kappa from 1.6 to 15, Sec. 5).
  C3  differentiation: 2^26 particles, kappa 2.5, theta 1.3, FP32 with FP64
      tail; upstream gradient dLoss/dv ~ N(0, 1) per component, seed 2.
  C4  batched PIC initialisation: 4096 cells x 3 species; counts lognormal
      (mu = ln 256, sigma = 1) rounded and clipped to [1, 8192]; per-species
      kappa ~ U[1.6, 10], theta ~ U[0.5, 2]; per-cell drift ~ N(0, 0.1^2) per
      axis; drawn with numpy default_rng(4); sampler seed 4.  Particles per
      cell of 1e2-1e3 follow the paper's remark on PIC codes (Sec. 6).
  C5  precision/tail stress: 1e9 particles, kappa 1.6, theta 1, streamed in
      chunks of 2^28 through counter_offset; seed 5.
"""
import numpy as np

C1 = dict(name="C1", n=10 ** 6, kappa=3.0, theta=1.0, seed=0)
C2 = dict(name="C2", n=10 ** 8, kappas=(1.6, 2.0, 3.0, 4.0, 6.0, 10.0), theta=1.0, seed=1)
C3 = dict(name="C3", n=1 << 26, kappa=2.5, theta=1.3, seed=2, grad_seed=2)
C4 = dict(name="C4", cells=4096, species=3, table_seed=4, seed=4, mu=float(np.log(256.0)), sigma=1.0,
          count_min=1, count_max=8192, kappa_range=(1.6, 10.0), theta_range=(0.5, 2.0), drift_sigma=0.1)
C5 = dict(name="C5", n=10 ** 9, chunk=1 << 28, kappa=1.6, theta=1.0, seed=5)


def batched_segments(cells=C4["cells"], species=C4["species"], table_seed=C4["table_seed"]):
    """C4 segment table as a list of dicts (kappa, theta, drift, count, seg_id),
    cell-major: seg_id = species * cell + s."""
    rng = np.random.default_rng(table_seed)
    kappas = rng.uniform(*C4["kappa_range"], size=species)
    thetas = rng.uniform(*C4["theta_range"], size=species)
    drifts = rng.normal(0.0, C4["drift_sigma"], size=(cells, 3))
    counts = rng.lognormal(mean=C4["mu"], sigma=C4["sigma"], size=cells * species)
    counts = np.clip(np.rint(counts), C4["count_min"], C4["count_max"]).astype(np.int64)
    segs = []
    for c in range(cells):
        for s in range(species):
            sid = species * c + s
            segs.append(dict(kappa=float(kappas[s]), theta=float(thetas[s]),
                             drift=tuple(float(d) for d in drifts[c]), count=int(counts[sid]), seg_id=sid))
    return segs


def batched_cells(cells=C4["cells"], species=C4["species"], grid=(16, 16, 16), spacing=(0.5, 0.5, 0.5),
                  origin=(-4.0, -4.0, -4.0)):
    """Cell boxes for the C4 segments, in segment order: cell c sits at
    (c % nx, (c // nx) % ny, c // (nx ny)) of a regular grid of spacing dx
    (16^3 = 4096 cells of 0.5^3 from -4); every species of a cell shares
    its box.  Array of shape (cells * species, 2, 3): (lo, size)."""
    nx, ny, _ = grid
    out = np.empty((cells * species, 2, 3))
    for c in range(cells):
        idx = np.array([c % nx, (c // nx) % ny, c // (nx * ny)], dtype=np.float64)
        lo = np.asarray(origin) + idx * np.asarray(spacing)
        for s in range(species):
            out[species * c + s, 0] = lo
            out[species * c + s, 1] = spacing
    return out


def upstream_gradient(n, seed=C3["grad_seed"]):
    """dLoss/dv ~ N(0, 1) per component: float32 array of shape (3, n)."""
    return np.random.default_rng(seed).standard_normal((3, n), dtype=np.float32)


def c5_chunks(n=C5["n"], chunk=C5["chunk"]):
    """(counter_offset, count) of each chunk of the C5 stream."""
    return [(off, min(chunk, n - off)) for off in range(0, n, chunk)]
