"""MI355X (gfx950) superquadric volume renderer (SQOcc-R, arXiv 2511.17361).

The compute path is the HIP library libsqr.so behind the C ABI of
include/sqr.h; `api` and `autograd` are thin torch bindings of it.
Submodules are imported lazily so that `import paper_2511_17361_amd` needs
neither torch nor a GPU."""

__all__ = ["api", "autograd", "build"]
