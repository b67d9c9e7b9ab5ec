"""strokex: GPU-friendly stroke expansion (Levien & Uguray, arXiv:2405.00127)
as a HIP library for AMD Instinct MI355X (gfx950).

``binding`` wraps the C ABI of ``libstrokex.so`` (include/strokex.h);
``scenes`` generates seeded synthetic inputs.
"""
__all__ = ["binding", "scenes"]
