"""MI355X (gfx950) steady phonon BTE-RTA transport library: HIP kernels behind
a C ABI (include/nbte.h), with a ctypes binding in `nbte`."""
