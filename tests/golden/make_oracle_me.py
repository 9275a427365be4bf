"""Writes oracle results for the GPU parity tests at the benchmark sizes.

    python tests/golden/make_oracle_me.py [--threads N] [--what me calib select] [--only NAME ...]

Only the oracle is called.  Every input is regenerated from its seed by the
oracle's own RAMBO (Philox4x32-10, sqrt(s) = 1500 GeV) or by a seeded numpy
generator, so the GPU tests rebuild the same inputs and compare the device
path with these values element by element.

  me:     oracle_me_<name>_<n>.npy, [n, 2] float64: |M|^2 of events 0 .. n-1
          of seed 230318244 in double (column 0) and in long double rounded
          to double (column 1).
  calib:  oracle_me_hel_gg_ttggg_calib64.npy, [64, 128] float64: the
          per-helicity |M_h|^2 of the 64 helicity-calibration events (seed 1)
          of g g -> t t~ g g g, from which the good-helicity list follows.
  select: oracle_select_gg_ttggg_1024.npy, [1024, 4] float64: helicity code,
          colour flow and the two margins of the oracle's helicity and
          leading-colour choice for events 0 .. 1023 of seed 230318244, with
          r_hel, r_col = numpy default_rng(77).random(1024) twice.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

SEED = 230318244
SQRT_S = 1500.0
WORKLOADS = {"gg_ttgg": 65536, "gg_ttggg": 8192}
N_SELECT = 1024
SELECT_RNG = 77


def path(name: str, n: int) -> str:
    return os.path.join(HERE, f"oracle_me_{name}_{n}.npy")


CALIB_PATH = os.path.join(HERE, "oracle_me_hel_gg_ttggg_calib64.npy")
SELECT_PATH = os.path.join(HERE, f"oracle_select_gg_ttggg_{N_SELECT}.npy")


def events(name: str, n: int, seed: int = SEED) -> np.ndarray:
    pdg = oracle.PROCESSES[name]
    masses = [173.0 if abs(x) == 6 else 0.0 for x in pdg[2:]]
    mom, _ = oracle.rambo(masses, SQRT_S, seed, 0, n)
    return mom


def select_randoms(n: int = N_SELECT):
    rng = np.random.default_rng(SELECT_RNG)
    return rng.random(n), rng.random(n)


def write_me(threads: int, only=None) -> None:
    for name, n in WORKLOADS.items():
        if only and name not in only:
            continue
        mom = events(name, n)
        P = oracle.Process(oracle.PROCESSES[name])
        t0 = time.time()
        d = P.me(mom, nthreads=threads)
        t1 = time.time()
        ld = P.me(mom, precision=1, nthreads=threads)
        t2 = time.time()
        np.save(path(name, n), np.stack([d, ld], axis=1))
        rel = np.abs(d / ld - 1.0)
        print(f"{name}: {n} events, double {t1 - t0:.0f} s, long double {t2 - t1:.0f} s; "
              f"double vs long double max rel {rel.max():.2e}", flush=True)


def write_calib(threads: int) -> None:
    mom = events("gg_ttggg", 64, seed=1)
    P = oracle.Process(oracle.PROCESSES["gg_ttggg"])
    with cf.ThreadPoolExecutor(threads) as ex:  # the oracle call releases the interpreter lock
        rows = list(ex.map(P.me_hel, mom))
    np.save(CALIB_PATH, np.array(rows))
    print(f"calibration: {len(rows)} events x {len(rows[0])} helicities", flush=True)


def write_select(threads: int) -> None:
    mom = events("gg_ttggg", N_SELECT)
    r_hel, r_col = select_randoms()
    P = oracle.Process(oracle.PROCESSES["gg_ttggg"])

    def one(e):
        h, c, margin = P.select(mom[e], float(r_hel[e]), float(r_col[e]))
        return [h, c, margin[0], margin[1]]

    with cf.ThreadPoolExecutor(threads) as ex:
        rows = list(ex.map(one, range(N_SELECT)))
    np.save(SELECT_PATH, np.array(rows, dtype=np.float64))
    print(f"select: {N_SELECT} events", flush=True)


def main(argv=None) -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--what", nargs="*", default=["me", "calib", "select"])
    ap.add_argument("--only", nargs="*", default=None, help="workloads of --what me")
    a = ap.parse_args(argv)
    for what in a.what:
        if what == "me":
            write_me(a.threads, a.only)
        else:
            {"calib": write_calib, "select": write_select}[what](a.threads)


if __name__ == "__main__":
    main()
