"""MI355X-native JaTAM assembly and classification (arXiv 2205.15311).

The work is done by the HIP library libjatam.so (include/jatam.h); this
package only binds it.
"""
from .jatam import (CLASS_NAMES, DET, GA, INVALID, MLP, ND_RUNS, ND_SITE,  # noqa: F401
                    PREDICT_COST, PREDICT_P_UNBOUND, PREDICT_SCREEN, UNBOUND, UNDECIDED,
                    VARIANT_C4, VARIANT_LIFO, Batch,
                    GAParams, JatamError, RouletteParams, Screen, Truth, Tuning, abi_version,
                    classify, classify_range, classify_static, classify_variant, fujiyama, ga_offspring, lib,
                    make_items, mutant_count, neighbourhood, neighbourhood_space, order_by_cost,
                    records_to_numpy, roulette_offspring, shape_histogram, shape_table_to_numpy,
                    single_mutants, strerror)
