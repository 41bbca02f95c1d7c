"""GS(p) geometric scaling + restarted GMRES(m) / Bi-CGSTAB on one MI355X (gfx950).

D. Gordon, R. Gordon, "Geometric scaling: a simple preconditioner for certain linear systems
with discontinuous coefficients" (2009).

  paper_0812_2769_amd.gsk       ctypes binding of libgsk.so (the C ABI in include/gsk.h);
                                importing it loads the HIP library and fails if it is absent
  paper_0812_2769_amd.problems  seeded synthetic convection-diffusion systems
  paper_0812_2769_amd.build     hipcc build of libgsk.so
"""

__all__ = ["gsk", "problems", "build"]


def __getattr__(name):
    if name in __all__:
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
