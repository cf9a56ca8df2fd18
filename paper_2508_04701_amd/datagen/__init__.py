"""Seeded synthetic workloads for the relational hot path.

Input plumbing only: this module draws columns and holds none of the
relational method's arithmetic. The oracle tests and the GPU path both take
their inputs from here. The paper measures on TPC-H and ClickBench
(Section 4.1); those datasets are not used. These generators stand in for
them with a star schema of the same flavour (a large fact table filtered on a
date range and joined to small dimension tables) and with join/group-by
stress inputs.

Draws are counter based (SplitMix64 + Lemire mapping, see ``gen.c``), so a
(seed, column) pair always yields the same bytes whatever the thread count.
Workload k uses seed ``SEED0 + k`` by default.
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

SEED0 = 2508047010

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB_PATH = os.path.join(_HERE, "libreldatagen.so")
_lib = None


def build() -> str:
    """Compiles gen.c (host C, OpenMP) into libreldatagen.so."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", "-o", _LIB_PATH + ".tmp",
           _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    U64, I64, P, I, D = ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.gen_splitmix64_at.restype = U64
    lib.gen_splitmix64_at.argtypes = [U64, U64]
    lib.gen_u64.argtypes = [U64, U64, I64, P]
    lib.gen_uniform.argtypes = [U64, U64, I64, I64, I64, P, I]
    lib.gen_permutation_i32.argtypes = [U64, U64, I64, P]
    lib.gen_unique_i64.argtypes = [U64, U64, I64, I64, P]
    lib.gen_map_ranks_i64.argtypes = [U64, U64, I64, I64, P, P]
    lib.gen_zipf.argtypes = [U64, U64, I64, D, I64, P]
    _lib = lib
    return lib


# ----------------------------------------------------------------- primitives

def splitmix64_at(s: int, i: int) -> int:
    """Output i (0-based) of the SplitMix64 sequence seeded with s."""
    return int(_load().gen_splitmix64_at(s & (2**64 - 1), i))


def raw_u64(seed: int, stream: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    _load().gen_u64(seed, stream, n, out.ctypes.data)
    return out


def uniform(seed: int, stream: int, lo: int, hi: int, n: int, dtype) -> np.ndarray:
    """n draws uniform over the integers [lo, hi)."""
    dtype = np.dtype(dtype)
    out = np.empty(n, dtype=dtype)
    _load().gen_uniform(seed, stream, lo, hi, n, out.ctypes.data, dtype.itemsize)
    return out


def permutation(seed: int, stream: int, n: int) -> np.ndarray:
    """A seeded permutation of 0..n-1 as int32."""
    out = np.empty(n, dtype=np.int32)
    _load().gen_permutation_i32(seed, stream, n, out.ctypes.data)
    return out


def unique_i64(seed: int, stream: int, n: int, first: int = 0) -> np.ndarray:
    """n distinct int64 values (a bijective mix of first..first+n-1)."""
    out = np.empty(n, dtype=np.int64)
    _load().gen_unique_i64(seed, stream, first, n, out.ctypes.data)
    return out


def map_ranks(seed: int, stream: int, m: int, ranks: np.ndarray) -> np.ndarray:
    """rank r -> mix((r - 1) mod m); with the same (seed, stream) and m = n this is
    ``unique_i64(seed, stream, n)[r - 1]``."""
    ranks = np.ascontiguousarray(ranks, dtype=np.int64)
    out = np.empty(len(ranks), dtype=np.int64)
    _load().gen_map_ranks_i64(seed, stream, m, len(ranks), ranks.ctypes.data, out.ctypes.data)
    return out


def zipf_ranks(seed: int, stream: int, N: int, theta: float, n: int) -> np.ndarray:
    """n Zipf(theta) ranks over 1..N (P(r) proportional to r^-theta)."""
    out = np.empty(n, dtype=np.int64)
    _load().gen_zipf(seed, stream, N, theta, n, out.ctypes.data)
    return out


# ----------------------------------------------------------------- workloads

def join_groupby(seed: int = SEED0 + 1, n_build: int = 65_536, n_probe: int = 1_048_576,
                 n_groups: int = 64, probe_domain: int = 72_090) -> dict:
    """Single inner join + group-by: build keys are a permutation of
    0..n_build-1 with a uniform group attribute; probe keys are uniform over
    0..probe_domain-1 (with 65,536 build keys and 72,090 values, 9.09% of
    probe rows find no partner); probe values uniform over [0, 1e6)."""
    return dict(
        build_key=permutation(seed, 1, n_build),
        build_grp=uniform(seed, 2, 0, n_groups, n_build, np.int32),
        probe_key=uniform(seed, 3, 0, probe_domain, n_probe, np.int32),
        probe_val=uniform(seed, 4, 0, 1_000_000, n_probe, np.int64),
    )


def star_schema(seed: int = SEED0 + 2, n_fact: int = 600_000_000, n_dim_a: int = 1_500_000,
                n_dim_b: int = 10_000, n_regions: int = 25, n_dates: int = 2557,
                n_cities: int = 5_000, n_segments: int = 1_000_000, attributes: bool = False) -> dict:
    """Star schema: fact(fk_a, fk_b, date, price, flag) with foreign keys
    uniform over the dim key ranges (so every fact row finds its dim rows),
    date uniform over [0, n_dates), price an int64 fixed-point x100 value
    uniform over [100, 1e7), flag uniform over {0, 1, 2}. Dim keys are seeded
    permutations of 0..n-1 in shuffled row order. Dim B carries region
    (uniform over n_regions values); with ``attributes`` dim B also carries
    city (a permutation mod n_cities) and dim A carries segment (a
    permutation mod n_segments)."""
    d = dict(
        fk_a=uniform(seed, 10, 0, n_dim_a, n_fact, np.int32),
        fk_b=uniform(seed, 11, 0, n_dim_b, n_fact, np.int32),
        date=uniform(seed, 12, 0, n_dates, n_fact, np.int32),
        price=uniform(seed, 13, 100, 10_000_000, n_fact, np.int64),
        flag=uniform(seed, 14, 0, 3, n_fact, np.int8),
        dim_a_key=permutation(seed, 20, n_dim_a),
        dim_b_key=permutation(seed, 21, n_dim_b),
        dim_b_region=uniform(seed, 22, 0, n_regions, n_dim_b, np.int32),
    )
    if attributes:
        d["dim_b_city"] = (permutation(seed, 23, n_dim_b) % n_cities).astype(np.int32)
        d["dim_a_segment"] = (permutation(seed, 24, n_dim_a) % n_segments).astype(np.int32)
    return d


def skewed(seed: int = SEED0 + 3, n_build: int = 100_000_000, n_probe: int = 400_000_000,
           n_groups: int = 10_000_000, theta: float = 1.0) -> dict:
    """High-cardinality, skewed join + group-by. Build keys are n_build
    distinct int64 values; probe row i draws a Zipf(theta) rank r over
    1..n_build and takes the key of build row r-1, so every probe row
    matches exactly once. The probe-side group column is a function of the
    rank, mix((r-1) mod n_groups), so the skew carries over to the groups;
    payload is uniform over [0, 1e6)."""
    ranks = zipf_ranks(seed, 30, n_build, theta, n_probe)
    d = dict(
        build_key=unique_i64(seed, 31, n_build),
        probe_key=map_ranks(seed, 31, n_build, ranks),
        probe_grp=map_ranks(seed, 32, n_groups, ranks),
        probe_val=uniform(seed, 33, 0, 1_000_000, n_probe, np.int64),
    )
    del ranks
    return d


def batch_shapes(seed: int = SEED0 + 4, n_inst: int = 256, build_range=(1_000, 4_000_000),
                 probe_range=(10_000, 50_000_000), group_range=(8, 100_000)) -> list:
    """Sizes of the batched instances: build rows, probe rows and group
    counts each log-uniform over their range (natural-log space, rounded);
    the group count is capped at the build size."""
    def logu(stream, lo, hi):
        u = raw_u64(seed, stream, n_inst).astype(np.float64) * 2.0 ** -64
        return np.rint(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)

    nb = logu(40, *build_range)
    npr = logu(41, *probe_range)
    ng = np.minimum(logu(42, *group_range), nb)
    return [dict(n_build=int(nb[i]), n_probe=int(npr[i]), n_groups=int(ng[i])) for i in range(n_inst)]


def batch_instance(seed: int, i: int, n_build: int, n_probe: int, n_groups: int,
                   match_rate: float = 0.9) -> dict:
    """One batched instance: build keys a permutation of 0..n_build-1 with a
    group attribute uniform over n_groups values; probe keys uniform over
    [0, ceil(n_build / match_rate)) so about match_rate of probes match;
    values uniform over [0, 1e6). Instance seed = seed xor i."""
    s = seed ^ i
    dom = int(math.ceil(n_build / match_rate))
    return dict(
        build_key=permutation(s, 50, n_build),
        build_grp=uniform(s, 51, 0, n_groups, n_build, np.int32),
        probe_key=uniform(s, 52, 0, dom, n_probe, np.int32),
        probe_val=uniform(s, 53, 0, 1_000_000, n_probe, np.int64),
    )
