"""MI355X-native JaTAM assembly and classification (arXiv 2205.15311).

The work is done by the HIP library libjatam.so (include/jatam.h); this
package only binds it.
"""
from .jatam import (CLASS_NAMES, DET, GA, INVALID, MLP, ND_RUNS, ND_SITE, UNBOUND,  # noqa: F401
                    UNDECIDED, PREDICT_COST, PREDICT_P_UNBOUND, PREDICT_SCREEN, Batch, GAParams, JatamError, Screen, Tuning, abi_version, classify,
                    classify_range, classify_static, ga_offspring,
                    lib, make_items, order_by_cost, records_to_numpy, shape_histogram,
                    shape_table_to_numpy, strerror, Truth)
