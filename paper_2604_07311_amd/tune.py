"""Write a tile table for this device with the library's autotuner.

    python -m paper_2604_07311_amd.tune --out PATH [--quick] [--batch-only | --plain-only]

famlies_tune times the candidate tiles on the device (plain kernels: tile
and split-K per size class; batched kernel: tile class per size class) and
writes one text line per size class; famlies_load_tune_table, or the
FAMLIES_TUNE_TABLE environment variable at handle creation, makes plans use
it.  Needs the GPU."""
import argparse
import time

import paper_2604_07311_amd as fm


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--device", type=int, default=0)
    ap.add_argument("--quick", action="store_true")
    g = ap.add_mutually_exclusive_group()
    g.add_argument("--batch-only", action="store_true")
    g.add_argument("--plain-only", action="store_true")
    args = ap.parse_args()
    flags = (fm.FAMLIES_TUNE_QUICK if args.quick else 0) | \
        (fm.FAMLIES_TUNE_BATCH_ONLY if args.batch_only else 0) | \
        (fm.FAMLIES_TUNE_PLAIN_ONLY if args.plain_only else 0)
    h = fm.famlies_create(args.device)
    t0 = time.time()
    fm.famlies_tune(h, args.out, flags)
    fm.famlies_destroy(h)
    print("wrote %s in %.1f s" % (args.out, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
