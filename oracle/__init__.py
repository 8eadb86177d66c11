"""Plain, slow CPU oracle for the DWT-fragmentation protect/restore path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_1803_04880_amd``) never imports it and shares no code with it.

Source: Qiu Han, "An Efficient Data Protection Architecture Based on
Fragmentation and Encryption" (arXiv 1803.04880), Chapter 5 (LeGall 5/3 lifting
DWT, fragment selection) and Chapter 2 section "Our SE approach" / "Performance
issue of SE" (AES-128 on the private fragment, counter mode as the parallel
mode).  Every function cites the passage it follows.

Modules
  dwt53     1-D / 2-D / multi-level integer 5/3 lifting, forward and inverse.
  aes128    AES-128 (S-box derived from GF(2^8) inversion + affine map), CTR.
  fragment  byte buffer -> matrix view -> fragments (priv, pub) and back.
  direct53  brute-force pointwise twin of dwt53 (nested-floor closed form,
            explicit mirror indexing, no shared intermediates), used only to
            pin dwt53 in tests.
  learned   learned context-MLP predictor variant of the lifting predict step
            (integer forward, fp64 training gradients).
  sha2      SHA-256 / SHA-512 (FIPS 180-4, constants derived from prime roots).
  se8       the thesis's per-8x8-block protection (Ch. 5 section 5.2.1):
            2-level block lifting, SHA keystreams XORed over the public
            fragments, 10/11-bit packed records, AES-CTR private fragment.
"""
