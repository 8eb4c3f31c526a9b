"""dagrt: a runtime DAG scheduler for GPU kernel and copy calls on MI355X.

Submodules (imported on demand so that the input generators can be used
without loading the native library):

``dagrt``      ctypes binding of the C-ABI in ``include/dagrt.h``
``workloads``  seeded synthetic inputs and the task programs of the
               benchmark workloads (pure data, none of the method's math)
``runner``     submits a workload program through the binding
``metrics``    critical-path bound and overlap metrics over task intervals
``build``      compiles the HIP library for gfx950
"""
