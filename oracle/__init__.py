"""Plain CPU oracle for the three-party protocol over Z_{2^64} (arXiv 2411.09287).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the HIP library; the two meet only
in the seeded input generators (``paper_2411_09287_amd/workloads.py``), which
hold no arithmetic of the method.

Modules
  ring      -- Z_{2^64} helpers, fixed-point encoding (Preliminaries, "Notation")
  gr        -- Galois ring Z_{2^64}[x]/f(x) (Sec. 3, "Ring-Specific Challenges")
  prg       -- ChaCha20 (RFC 8439) keystream standing in for the pairwise-seed PRG
  protocol  -- the parties' steps: sharing, Pi_Inner, Pi_Mult, Pi_Trunc, Pi_Rec,
               Pi_Tran / Pi_Reduce / Pi_InnerVerify / Pi_MultVerify / Pi_BIVerify

Everything is in uint64 numpy arithmetic, which wraps modulo 2^64 exactly.
Parity of the exact intermediate verification values (h(0), h(2), zeta, the
mask words, Delta shares) is *unpinned* by the paper, which prints no worked
example; those are pinned only by their invariants (see protocol.py).
"""
