"""FP64 CPU oracle of the shear 4PCF multipole estimator.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``; never by the library.
"""
from .estimator import (NCORR, FACTORS, TABLE1, family_orders, squared_edges,
                        centre_neighbours, bin_counts, centre_multipoles,
                        multipoles, contract, upsilon, upsilon_parallel, abs_bound,
                        abs_bound_parallel, contract_triplets, upsilon_triplets,
                        upsilon_triplets_parallel)
from .brute import brute_upsilon, brute_angular_bins
from .natural import (angular_integrals, binned_from_multipoles, natural_components,
                      natural_components_triplets, natural_components_selected)
from .nthorder import (beta_matrix, arg_coefficients, norm_coefficients, upsilon_n, upsilon3,
                       brute_upsilon3)
from .tree import (tree_levels, reduced_catalogue, reduced_hierarchy, tree_centre_multipoles,
                   upsilon_tree, brute_tree_upsilon)
