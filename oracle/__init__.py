"""Plain, slow FP64 CPU oracle for the block-FSAI / fourth-kind Chebyshev path.

TEST INFRASTRUCTURE ONLY. Nothing in the product path (the package
``paper_2509_06744_amd`` and its HIP library) may import, call or execute
anything here; only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` use it. It shares no code with the HIP path: the only common
dependency is the seeded input generator in ``problems/``.

Each function follows a passage of the paper (cited in its docstring) written
out in NumPy/SciPy in double precision, with no blocking, fusion or reordering
beyond what the definition or algorithm states.

Readings of the paper where it is silent, ambiguous or garbled (restated in the
design notes):
  * block indices are 0-based; admissible candidates are c < k;
  * W_k(1) = 2k+1 (the Remark after Lemma 3.2 prints the reciprocal);
  * S^{-1/2} is taken as the inverse Cholesky root J = L_S^{-1} (S = L_S L_S^T);
  * "H_kc not identically zero" is read structurally (pattern of F_k A);
  * ties in argmin rho_c are broken by a relative window of 1e-9 on
    g = -log rho_c followed by the smallest block index;
  * with tau = 1 a candidate is added when g* > -log(tau) + 1e-12.

Functions without an independent pin say "parity unpinned" in their docstring.
"""
