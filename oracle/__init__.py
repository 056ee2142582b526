"""Plain CPU oracle for the Pauli-sum operator-state path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the ``paper_2606_28952_amd``
package and its HIP library) may import, call or link anything here; only the
tests, the smoke check of the build entry point and the CPU-baseline leg of
the benchmark use it.

Every function is written from the definitions in the paper (arxiv
2606.28952, "A High-Performance Pauli-Algebra Framework for Large-Scale
Quantum Simulations") in float64 and plain NumPy, deliberately slow and
obviously correct.  It shares no code, table or helper with the HIP path:

* Pauli products use the single-qubit letter table (sigma_a sigma_b =
  delta_ab I + i eps_abc sigma_c) position by position, not the symplectic
  XOR/popcount rule of Section 2.3 that the library implements.
* Canonical reduction sums each key's coefficients with ``math.fsum``
  (a documented correctly-rounded summation), then sorts with ``np.lexsort``.
* Jordan-Wigner goes the "conventional" way mentioned in Section 2.3: each
  ladder operator is a two-term Pauli sum, the sums are multiplied and the
  product is reduced, instead of Algorithm 1's precomputed 4/16 expansions.
* Sector indexing ranks a spin string by its position in the explicitly
  enumerated ascending list, not by a combinatorial formula.
* Operator application scatters term by term over source configurations,
  the plain definition behind Eq. grouped_contraction, while the kernels
  gather per X-mask group (Eq. reverse_sum).  ``capply.c`` (loaded by
  ``native``) is a plain C float64 twin of that scatter and of the ungrouped
  per-target gather, threaded with OpenMP, for full-size workloads; it
  ranks sector configurations through position tables built from the
  enumerated spin strings.

Readings of points the paper leaves open are listed in the module that uses
them and in the design notes of the repository.
"""
