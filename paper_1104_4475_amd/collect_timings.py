"""Collect the selector's timing data on the current GPU.

  python -m paper_1104_4475_amd.collect_timings corpus OUT.csv --count 5000 --seed 11
      random candidates (training corpus), columns p,q,nb,algo,kern,bs,prec,ms
  python -m paper_1104_4475_amd.collect_timings heldout OUT.csv --count 200 --seed 12 [--first i --last j]
      exhaustive autotuner tables of held-out shapes, columns
      shape,m,n,prec,nb,algo,kern,bs,ms

Times are the executor kernel's duration (HIP events) of one factorization
after one warm-up run on the same handle.
"""

import argparse
import csv
import os
import sys

from . import selector


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["corpus", "heldout"])
    ap.add_argument("out")
    ap.add_argument("--count", type=int, default=100)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--first", type=int, default=0)
    ap.add_argument("--last", type=int, default=None)
    a = ap.parse_args(argv)

    def log(msg):
        print("%s %s" % (selector.now(), msg), flush=True)

    if a.what == "corpus":
        selector.collect_corpus(a.out, a.count, seed=a.seed, log=log)
        return 0
    shapes = selector.heldout_shapes(a.count, a.seed)
    last = a.count if a.last is None else min(a.last, a.count)
    timer = selector.Timer(a.seed)
    new = not os.path.exists(a.out)
    with open(a.out, "a", newline="") as fh:
        w = csv.writer(fh)
        if new:
            w.writerow(["shape", "m", "n", "prec", "nb", "algo", "kern", "bs", "ms"])
        for s in range(a.first, last):
            m, n, prec = shapes[s]
            table = selector.exhaustive(m, n, prec, timer)
            for (nb, algo, kern, bs), ms in table.items():
                w.writerow([s, m, n, prec, nb, algo, kern, bs, "%.5f" % ms])
            fh.flush()
            log("shape %d: %d x %d prec %d, %d candidates" % (s, m, n, prec, len(table)))
    return 0


if __name__ == "__main__":
    sys.exit(main())
