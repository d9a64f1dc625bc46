"""airhip: the AIRLab (arXiv 1806.09907) registration objective and gradient
as hand-written HIP kernels for the AMD Instinct MI355X (gfx950).

Import `paper_1806_09907_amd.api` for the C-ABI binding; this package
initialiser loads nothing by itself.
"""
__all__ = ["api", "autograd", "synth", "build"]
