"""Traffic and flop model of the multi-RHS Wilson stencil.

Paper's accounting (Sec. 2.1): eta_x costs 1320 flops and 360 words per site
for one right-hand side: 8 neighbour spinors (8 x 24 words) loaded, 24 words
stored and 8 links (8 x 18 words) loaded.  With L right-hand sides sharing
the links (block hopping-term equation), spinor words scale with L and link
words do not: 216 L + 144 words.  The O(a)-improved (clover) operator adds a
site-diagonal 2 x (6x6 Hermitian) term: +72 words per site, +504 flops per
site and right-hand side; Fig. 1 plots flops/byte of both in single precision.

Compulsory (algorithmic) traffic of one application A X on the whole lattice,
each array touched exactly once: read and write the L spinors (2 x 24 L
words) and read the 4 forward links of every site (72 words), i.e.
(48 L + 72) words per site.  The FP16-storage format keeps 24 halves plus
one FP32 scale per (site, column) and 72 halves of links: 104 L + 144 bytes.

Flops per site and right-hand side: 1320 for eta plus 48 for phi - kappa*eta.
"""

WILSON_FLOPS = 1320
CLOVER_EXTRA_FLOPS = 504
CLOVER_EXTRA_WORDS = 72
AXPY_FLOPS = 48

WORD = {"fp64": 8, "fp32": 4}


def paper_words_per_site(L: int, clover: bool = False) -> int:
    return 216 * L + 144 + (CLOVER_EXTRA_WORDS if clover else 0)


def paper_flops_per_site(L: int, clover: bool = False) -> int:
    return (WILSON_FLOPS + (CLOVER_EXTRA_FLOPS if clover else 0)) * L


def paper_flops_per_byte(L: int, word_bytes: int, clover: bool = False) -> float:
    return paper_flops_per_site(L, clover) / (paper_words_per_site(L, clover) * word_bytes)


def link_bytes_per_site(word_bytes: int) -> int:
    """The 8 links touching a site (4 forward, 4 backward), Sec. 2.1."""
    return 8 * 18 * word_bytes


def dslash_bytes_per_site(L: int, prec: str, clover: bool = False) -> int:
    """Compulsory HBM bytes of one full-lattice application, per site; with
    the clover term also the packed site inverse (72 reals, FP32 for the
    FP16-storage operator)."""
    cl = 72 * (8 if prec == "fp64" else 4) if clover else 0
    if prec == "fp16s":
        return 104 * L + 144 + cl
    return (48 * L + 72) * WORD[prec] + cl


def dslash_flops_per_site(L: int) -> int:
    return (WILSON_FLOPS + AXPY_FLOPS) * L
