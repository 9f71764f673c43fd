"""Shared test helpers: fixture loading and field-by-field record comparison."""
import json
import os

import numpy as np

from paper_1308_4011_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_fixture(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def fixture_system(fx, variant=None):
    src = fx if variant is None else {**fx, **fx[variant]}
    return synth.from_lists(fx["n_classes"], src["method_class"], fx["attr_class"],
                            src["acc_rows"], src["call_rows"])


def assert_fields_equal(a, b, fields, what=""):
    for f in fields:
        x = np.asarray(a[f])
        y = np.asarray(b[f])
        if not np.array_equal(x, y):
            bad = np.nonzero(x != y)[0][:10]
            raise AssertionError(f"{what} field {f!r} differs at {bad.tolist()}: {x[bad].tolist()} vs {y[bad].tolist()}")


CLASS_FIELDS = ["n_methods", "n_attrs", "cbo", "rfc", "lcom_p", "lcom_q", "hs_num", "hs_den"]
METHOD_FIELDS = ["fan_in", "fan_out", "own_attr_uses", "own_coaccess_partners"]
MOVE_FIELDS = ["method", "src", "dst", "d_cbo_src", "d_cbo_dst", "d_rfc_src", "d_rfc_dst",
               "n_caller_cls", "n_caller_worse", "n_caller_better", "keep",
               "d_lcom_src", "d_lcom_dst", "hs_num_src", "hs_den_src", "hs_num_dst", "hs_den_dst"]


def oracle_score_threaded(sys_, cm, ct, mask, rule, threads=None):
    """The first oracle's records for many candidates, scored in slices on host
    threads (each slice is its own oracle call with no shared state; ctypes
    releases the interpreter lock during the call)."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle as O
    from oracle.incremental import host_threads
    nt = threads or host_threads()
    cm = np.asarray(cm)
    ct = np.asarray(ct)
    if len(cm) == 0:
        return O.score(sys_, cm, ct, mask, rule)
    parts = np.array_split(np.arange(len(cm)), min(nt * 4, len(cm)))
    with ThreadPoolExecutor(nt) as ex:
        outs = list(ex.map(lambda p: O.score(sys_, cm[p], ct[p], mask, rule), parts))
    return np.concatenate(outs)
