"""Synthetic workload recipes shaped like the paper's experiments.

The paper compares up to 2048 unknown profiles against up to 20 million known
ones (Section IV, abstract); its profiles are not available, so seeded
synthetic profiles with these shapes stand in for them:

* references: one bit per SNP locus (minor allele present), Bernoulli with a
  per-locus minor-allele frequency drawn uniformly from [maf_lo, 0.5);
* mixture queries: the OR of nc in [nc_lo, nc_hi] distinct references drawn
  from the database, then each bit flipped independently with probability
  ``flip``;
* identity queries: one reference from the database with the same flips.
"""
from __future__ import annotations

from dataclasses import dataclass

from . import MASTER_SEED


@dataclass(frozen=True)
class Workload:
    name: str
    n_q: int
    n_refs: int
    n_loci: int
    maf_lo: float
    nc_lo: int
    nc_hi: int
    flip: float
    mode: int  # 0 mixture (R AND NOT Q), 1 identity (XOR)
    seed: int
    k: int = 32

    @property
    def comparisons(self) -> int:
        """Query-ref-locus comparisons of one all-pairs pass."""
        return self.n_q * self.n_refs * self.n_loci


# 64 mixtures x 20,000 references x 2,048 loci, full count matrix.
MIX_64x20K = Workload("mixture-64x20000x2048-full", 64, 20_000, 2048, 0.05, 1, 4, 0.005, 0,
                      MASTER_SEED + 1)
# 2,048 mixtures x 20,000,000 references x 2,048 loci, top-32 (+ verification tiles).
MIX_2048x20M = Workload("mixture-2048x20Mx2048-top32", 2048, 20_000_000, 2048, 0.05, 1, 4,
                        0.005, 0, MASTER_SEED + 2)
# 256 mixtures x 2,000,000 references x 32,768 loci, threshold (<= 2% of loci) + top-32.
MIX_256x2Mx32K = Workload("mixture-256x2Mx32768-thr2pct-top32", 256, 2_000_000, 32768, 0.01,
                          2, 6, 0.01, 0, MASTER_SEED + 4)

BY_NAME = {w.name: w for w in (MIX_64x20K, MIX_2048x20M, MIX_256x2Mx32K)}


def scaled(w: Workload, n_q: int | None = None, n_refs: int | None = None,
           n_loci: int | None = None, name: str | None = None) -> Workload:
    """Same generator recipe at other sizes (parity cases the oracle can finish)."""
    return Workload(name or w.name + "-scaled", n_q or w.n_q, n_refs or w.n_refs,
                    n_loci or w.n_loci, w.maf_lo, w.nc_lo, w.nc_hi, w.flip, w.mode, w.seed, w.k)


def threshold_2pct(n_loci: int) -> int:
    """Count threshold '<= 2% of loci', read as floor(2 L / 100)."""
    return (2 * n_loci) // 100


# --------------------------------------------------------------------- ragged batches
# 400 independent top-32 jobs: query counts uniform in 1..512, reference
# slices of uniform length in 10k..2M taken from a 2M-reference pool per loci
# panel, panels drawn from {1024, 2048, 4096, 8192, 16384}, modes 50/50.
# Each panel pool uses the mixture generator above (MAF U(0.05, 0.5)); a
# mixture query ORs 1-4 references of its job's slice plus 0.5% flips, an
# identity query is one reference of the slice plus 0.5% flips.
RAGGED_PANELS = (1024, 2048, 4096, 8192, 16384)
RAGGED_SEED = MASTER_SEED + 3


@dataclass(frozen=True)
class RaggedJob:
    index: int
    n_q: int
    r_lo: int
    r_hi: int
    n_loci: int
    mode: int

    @property
    def q_row0(self) -> int:
        """First generator row of the job's queries (rows are unique per job)."""
        return self.index << 10

    @property
    def comparisons(self) -> int:
        return self.n_q * (self.r_hi - self.r_lo) * self.n_loci


def ragged_jobs(n_jobs: int = 400, seed: int = RAGGED_SEED, pool: int = 2_000_000,
                q_max: int = 512, r_min: int = 10_000, r_max: int = 2_000_000,
                panels=RAGGED_PANELS) -> list[RaggedJob]:
    from . import u64s
    r_max = min(r_max, pool)
    r_min = min(r_min, r_max)
    jobs = []
    for j in range(n_jobs):
        u = u64s(seed, 4, j, 5)
        n_q = 1 + int(u[0] % q_max)
        n_r = r_min + int(u[1] % (r_max - r_min + 1))
        L = panels[int(u[2] % len(panels))]
        mode = int(u[3] % 2)
        r_lo = int(u[4] % (pool - n_r + 1))
        jobs.append(RaggedJob(j, n_q, r_lo, r_lo + n_r, L, mode))
    return jobs


def ragged_panel_seed(seed: int, n_loci: int) -> int:
    return seed + n_loci


def ragged_queries(job: RaggedJob, thr, seed: int = RAGGED_SEED, flip: float = 0.005):
    """0/1 query bytes (n_q, L) of one ragged job."""
    from . import identity, mixtures
    ps = ragged_panel_seed(seed, job.n_loci)
    if job.mode == 0:
        return mixtures(ps, thr, job.r_lo, job.r_hi - job.r_lo, job.q_row0, job.n_q, 1, 4, flip)[0]
    return identity(ps, thr, job.r_lo, job.r_hi - job.r_lo, job.q_row0, job.n_q, flip)[0]
