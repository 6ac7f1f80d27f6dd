"""Plain FP64 CPU oracle for FRAM-RIR batched multi-channel RIR synthesis.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(the HIP library and its Python binding) never imports, calls or links anything
here, and nothing here imports the product.  The only module both sides share
is the seeded synthetic-input generator, which holds none of the method's
arithmetic.

Modules
-------
philox   Philox-4xW-10 counter-based generator, written from its publication.
cbrt     Correctly rounded FP64 cube root by exact integer arithmetic.
framrir  The method itself: room scalars (Eq. 2, 5), image draws (Sec. III-B,
         III-C, Eq. 3, 4, 6), band-limited rendering of Eq. 1 / Eq. 8, the
         adjoints with the draws held fixed and through the draws, finite
         differences, and the early-reverberation filter (Eq. 9).
multirate  The paper-literal rendering: high-rate impulses (Eq. 7, 8),
         down-sampling, the 80 Hz high-pass and the second down-sampling
         (Sec. II).
spatialize  Spatialisation and mixing of the training set-up (Sec. IV-A):
         each dry signal convolved with its RIRs, the second speaker scaled
         to the SIR and the noise to the SNR, the mixture as their sum.

Every function is slow and direct on purpose: there is no blocking, fusion or
reordering beyond what the paper's definitions state.
"""
