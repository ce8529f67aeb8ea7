"""Algorithmic (compulsory) byte and flop counts of the hop path.

Every array a kernel must touch is counted once per launch: each output
site reads its eight hop links (stored per output site, so there is no
reuse to be had), reads every input colour vector once (the eight-fold
neighbour reuse is the caches' job), reads the same-parity vectors its
epilogue needs and writes its output once. The paper counts one D per site
as 1584 bytes (8 links, 8 neighbour vectors and one output, fp64, no reuse)
and 576 flops (8 hops x 9 complex multiply-adds x 8 flops) (Sec.2, after
Eq.5); the flop convention is the paper's, the byte convention is the
compulsory one.

Bytes per stored link matrix / colour vector:
  f64  144 / 48   (12-parameter storage: 96 per link)
  f32   72 / 24   (12-parameter storage: 48 per link)
  f16s  36 (12-parameter: 24; + one 4-byte scale per site shared by its
        8 links) / 16

The improved operator (``improved=True``: fat links plus three-hop long
links) reads sixteen links per output site and does sixteen hops, so its
link bytes and D flops double; the vector bytes are unchanged (the extra
neighbours are again the caches' job).
"""

LINK_BYTES = {"f64": 144, "f32": 72, "f16s": 36}
# 12-parameter storage (two rows per SU(3) link)
LINK_BYTES_R12 = {"f64": 96, "f32": 48, "f16s": 24}
SPINOR_BYTES = {"f64": 48, "f32": 24, "f16s": 16}
SITE_SCALE_BYTES = {"f64": 0, "f32": 0, "f16s": 4}

FLOPS_PER_SITE_D = 576          # paper's count for one D at one site
FLOPS_PER_SITE_XPAY = 12        # m^2 x - t over 3 complex numbers
FLOPS_PER_SITE_DOT = 12         # Re<x, h> over 3 complex numbers


def hop_bytes_per_site(prec: str, stage: int, nrhs: int = 1, lazy: bool = False,
                       r12: bool = False, improved: bool = False) -> int:
    """Compulsory bytes per output site of one hop launch.

    stage 1 (D_oe, plain output): 8 links + nrhs x (read input + write output)
    stage 2 (D_eo, m^2 update + dot): 8 links + nrhs x (read t, read x, write)
    lazy (inside a CG iteration, the direction update d = r + beta d is
    formed in the kernel): stage 1 also reads r; stage 2 also reads r and
    writes the new d.
    """
    nlinks = 16 if improved else 8
    links = nlinks * (LINK_BYTES_R12 if r12 else LINK_BYTES)[prec] + SITE_SCALE_BYTES[prec]
    if stage == 1:
        nvec = 3 if lazy else 2
    else:
        nvec = 5 if lazy else 3
    return links + nrhs * nvec * SPINOR_BYTES[prec]


def a_bytes_per_site(prec: str, nrhs: int = 1, r12: bool = False, improved: bool = False) -> int:
    """One application of A = both stages, per even site."""
    return (hop_bytes_per_site(prec, 1, nrhs, r12=r12, improved=improved)
            + hop_bytes_per_site(prec, 2, nrhs, r12=r12, improved=improved))


def a_flops_per_site(nrhs: int = 1, improved: bool = False) -> int:
    d = 2 * FLOPS_PER_SITE_D if improved else FLOPS_PER_SITE_D
    return nrhs * (2 * d + FLOPS_PER_SITE_XPAY)


REAL_BYTES = {"f64": 8, "f32": 4, "f16s": 2}


def paper_d_bytes_per_site(prec: str = "f64", r12: bool = False, improved: bool = False) -> int:
    """Bytes of one D at one site in the paper's convention (Sec.2, after
    Eq.5: 1584 in fp64): every link and every neighbour vector read with no
    reuse, one output vector written; 18 reals per link (12 stored with
    12-parameter links), 6 per colour vector."""
    nhops = 16 if improved else 8
    reals = nhops * (12 if r12 else 18) + nhops * 6 + 6
    return reals * REAL_BYTES[prec]


def paper_a_bytes_per_site(prec: str = "f64", r12: bool = False, improved: bool = False) -> int:
    """One A (two D) per even site in the paper's convention."""
    return 2 * paper_d_bytes_per_site(prec, r12, improved)


def update_bytes_per_site(prec: str, mixed: bool) -> int:
    """Fused update: fp64 CG reads x, r, d, Ad and writes x, r; mixed reads
    y (fp32), rs, d, Ad and writes y, rs."""
    if not mixed:
        return 6 * SPINOR_BYTES["f64"]
    return 2 * SPINOR_BYTES["f32"] + 4 * SPINOR_BYTES[prec]


def cg_iteration_bytes_per_site(prec: str, mixed: bool, nrhs: int = 1, r12: bool = False,
                                improved: bool = False) -> int:
    """One CG iteration as run (three kernels: lazy stage 1, lazy stage 2, update)."""
    return (hop_bytes_per_site(prec, 1, nrhs, lazy=True, r12=r12, improved=improved)
            + hop_bytes_per_site(prec, 2, nrhs, lazy=True, r12=r12, improved=improved)
            + nrhs * update_bytes_per_site(prec, mixed))


def cg_iteration_flops_per_site() -> int:
    # A + <d,Ad> + 2 axpy + |r|^2 + the deferred xpay (paper-style count, 12 flops
    # per complex-vector op)
    return 2 * FLOPS_PER_SITE_D + FLOPS_PER_SITE_XPAY + 5 * 12
