"""ctypes binding of libdmpt.so (the C ABI in include/dmpt.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Loading fails loudly when the library has not been built.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdmpt.so")

DMPT_OK = 0
DMPT_ERR_ARG = -1
DMPT_ERR_HIP = -2
DMPT_ERR_NOMEM = -3
DMPT_ERR_NOCONV = -4
DMPT_ERR_RANGE = -5
DMPT_ERR_NONFINITE = -6
DMPT_ERR_UNSUPPORTED = -7

STATUS_NAMES = {
    DMPT_OK: "DMPT_OK", DMPT_ERR_ARG: "DMPT_ERR_ARG", DMPT_ERR_HIP: "DMPT_ERR_HIP",
    DMPT_ERR_NOMEM: "DMPT_ERR_NOMEM", DMPT_ERR_NOCONV: "DMPT_ERR_NOCONV",
    DMPT_ERR_RANGE: "DMPT_ERR_RANGE", DMPT_ERR_NONFINITE: "DMPT_ERR_NONFINITE",
    DMPT_ERR_UNSUPPORTED: "DMPT_ERR_UNSUPPORTED",
}

PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3, "int8x13": 4, "int8x6": 5}
SOLVER = {"cg": 0, "ns": 1, "hybrid": 2}
GUESS = {"prev": 0, "taylor": 1}
MAX_DIRS = 8


class Options(ctypes.Structure):
    _fields_ = [
        ("prec", ctypes.c_int), ("solver", ctypes.c_int), ("guess", ctypes.c_int),
        ("tol_occ", ctypes.c_double), ("tol_cg", ctypes.c_double),
        ("max_newton", ctypes.c_int), ("max_cg", ctypes.c_int), ("refine", ctypes.c_int),
        ("ckpt_every", ctypes.c_int), ("check", ctypes.c_int), ("staged", ctypes.c_int),
        ("warm_traj", ctypes.c_int), ("schedule", ctypes.c_int), ("acc64", ctypes.c_int),
        ("autotune", ctypes.c_int), ("grouped", ctypes.c_int),
    ]


FLAG_NOISE_FLOOR = 1
FLAG_CG_FLOOR = 2

_TRACES = ["tr_h1p1", "tr_h1p2", "tr_h2p0", "tr_h1p3", "tr_h1p0", "tr_h2p1", "tr_h2p2", "tr_h3p0",
           "tr_h3p1", "omega1", "omega2", "omega3", "omega4"]


class Stats(ctypes.Structure):
    _fields_ = [
        ("newton_iters", ctypes.c_int), ("cg_iters_total", ctypes.c_int),
        ("cg_iters_max", ctypes.c_int), ("flags", ctypes.c_int), ("cg_unconverged", ctypes.c_int),
        ("occ_err", ctypes.c_double),
        ("mu", ctypes.c_double * (1 + 3 * MAX_DIRS)), ("trP", ctypes.c_double * (1 + 3 * MAX_DIRS)),
        ("tr_pmu", ctypes.c_double),
    ] + [(name, ctypes.c_double * MAX_DIRS) for name in _TRACES] + [
        ("idempotency", ctypes.c_double), ("commutator", ctypes.c_double),
        ("asymmetry", ctypes.c_double), ("mfma_flops", ctypes.c_double),
        ("useful_flops", ctypes.c_double), ("seconds", ctypes.c_double),
    ]

    def as_dict(self, d=0, order=0):
        nmu = 1 + order * d
        out = dict(
            newton_iters=self.newton_iters, cg_iters_total=self.cg_iters_total,
            cg_iters_max=self.cg_iters_max, flags=self.flags, cg_unconverged=self.cg_unconverged,
            occ_err=self.occ_err, mu=list(self.mu[:nmu]), trP=list(self.trP[:nmu]), tr_pmu=self.tr_pmu,
            idempotency=self.idempotency,
            commutator=self.commutator, asymmetry=self.asymmetry, mfma_flops=self.mfma_flops,
            useful_flops=self.useful_flops, seconds=self.seconds)
        for name in _TRACES:
            out[name] = list(getattr(self, name)[:d])
        return out


class SparseStats(ctypes.Structure):
    _fields_ = [
        ("newton_iters", ctypes.c_int), ("block", ctypes.c_int),
        ("mu", ctypes.c_double * (1 + 2 * MAX_DIRS)), ("trP", ctypes.c_double * (1 + 2 * MAX_DIRS)),
        ("tr_h1p1", ctypes.c_double * MAX_DIRS), ("tr_h1p2", ctypes.c_double * MAX_DIRS),
        ("nnz_p0", ctypes.c_double), ("nnz_p1", ctypes.c_double * MAX_DIRS),
        ("nnz_p2", ctypes.c_double * MAX_DIRS), ("blocks_p0", ctypes.c_double),
        ("blocks_p1", ctypes.c_double * MAX_DIRS), ("blocks_p2", ctypes.c_double * MAX_DIRS),
        ("blocks_max", ctypes.c_double), ("block_products", ctypes.c_double), ("seconds", ctypes.c_double),
    ]

    def as_dict(self, d=0, order=0):
        nmu = 1 + order * d
        out = dict(newton_iters=self.newton_iters, block=self.block, mu=list(self.mu[:nmu]),
                   trP=list(self.trP[:nmu]), nnz_p0=self.nnz_p0, blocks_p0=self.blocks_p0,
                   blocks_max=self.blocks_max, block_products=self.block_products, seconds=self.seconds)
        for name in ("tr_h1p1", "tr_h1p2", "nnz_p1", "nnz_p2", "blocks_p1", "blocks_p2"):
            out[name] = list(getattr(self, name)[:d])
        return out


class ProfileData(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("mfma_flops", ctypes.c_double), ("useful_flops", ctypes.c_double),
                ("eng_launches", ctypes.c_int64 * 6), ("eng_ms", ctypes.c_double * 6),
                ("eng_mfma_flops", ctypes.c_double * 6), ("eng_bytes", ctypes.c_double * 6),
                ("eng_useful_flops", ctypes.c_double * 6)]


EXPORTS = [
    "dmpt_default_options", "dmpt_init", "dmpt_finalize", "dmpt_last_error", "dmpt_set_options",
    "dmpt_fermi_recursion", "dmpt_response", "dmpt_mu_newton", "dmpt_mu_newton_batched",
    "dmpt_backward", "dmpt_profile", "dmpt_profile_get", "dmpt_bench_product", "dmpt_autotune",
    "dmpt_congruence", "dmpt_fermi_recursion_noalloc", "dmpt_sparse_response", "dmpt_set_variant",
    "dmpt_get_variant",
]

_lib = None
P = ctypes.c_void_p
PP = ctypes.POINTER(ctypes.c_void_p)
I64 = ctypes.c_int64
D = ctypes.c_double
DP = ctypes.POINTER(ctypes.c_double)
I = ctypes.c_int


def load(path=None):
    """Load libdmpt.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} not found: build it with `python -m paper_1503_07037_amd.build`")
    lib = ctypes.CDLL(p)
    lib.dmpt_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.dmpt_default_options.restype = None
    lib.dmpt_init.argtypes = [ctypes.POINTER(P), I, I64, I, ctypes.POINTER(Options), P]
    lib.dmpt_finalize.argtypes = [P]
    lib.dmpt_last_error.argtypes = [P]
    lib.dmpt_last_error.restype = ctypes.c_char_p
    lib.dmpt_set_options.argtypes = [P, ctypes.POINTER(Options)]
    lib.dmpt_fermi_recursion.argtypes = [P, I64, P, D, D, I, P, ctypes.POINTER(Stats)]
    lib.dmpt_response.argtypes = [P, I64, P, I, PP, PP, PP, D, I, I, DP, P, PP, PP, PP,
                                  ctypes.POINTER(Stats)]
    lib.dmpt_mu_newton.argtypes = [P, I64, P, I, PP, PP, PP, D, D, I, I, DP, P, PP, PP, PP,
                                   ctypes.POINTER(Stats)]
    lib.dmpt_mu_newton_batched.argtypes = [P, I, ctypes.POINTER(I64), PP, I, PP, DP, DP, I, I, DP,
                                           PP, PP, PP, ctypes.POINTER(Stats)]
    lib.dmpt_backward.argtypes = [P, I64, P, D, D, I, DP, P, P, ctypes.POINTER(Stats)]
    lib.dmpt_profile.argtypes = [P, I]
    lib.dmpt_profile_get.argtypes = [P, ctypes.POINTER(ProfileData)]
    lib.dmpt_bench_product.argtypes = [P, I64, I, I, I, DP, DP]
    lib.dmpt_autotune.argtypes = [P, I64, ctypes.POINTER(I)]
    lib.dmpt_set_variant.argtypes = [P, I64, I, I]
    lib.dmpt_get_variant.argtypes = [P, I64, I, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.c_char_p, I]
    lib.dmpt_congruence.argtypes = [P, I64, P, P, P, I, ctypes.POINTER(Stats)]
    lib.dmpt_fermi_recursion_noalloc.argtypes = [I64, P, D, D, I, P, P, P]
    lib.dmpt_sparse_response.argtypes = [P, I64, P, I, PP, D, D, I, I, D, D, I, DP, P, PP, PP,
                                         ctypes.POINTER(SparseStats)]
    for name in EXPORTS:
        if name not in ("dmpt_default_options", "dmpt_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib
