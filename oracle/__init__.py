"""Oracle for the multi-particle aggregation right-hand side: TEST INFRASTRUCTURE.

Plain, slow, obviously correct CPU implementations of what the HIP path
computes, written from the paper (Stefonishin, Matveev, Zheltkov, "Tensors in
modelling multi-particle interactions"):

* ``rhs_direct``   literal O(N^D) sums of the operators p_k^(d), q_k^(d) (Sec. 1)
* ``rhs_conv``     the same sums regrouped per rank-one term as direct
                   truncated linear convolutions (Sec. 1, CP remark)
* ``rhs_fft``      the CP-FFT method of the Sec. 1 CP remark with numpy's FFT as a
                   library step, one product of spectra per (d, r)
* ``rhs_sum_kernel`` the definitions specialised to kernels that depend on the
                   total size only (no factorisation involved)
* ``rhs_factored`` the same method in C with its own FFT and OpenMP threads:
                   the factored CPU version GPU throughput is compared with
* ``heun_solve``   explicit second-order Runge-Kutta (Heun) time stepping (Sec. 3)
* closed forms     constant-kernel zeroth moment, binary constant kernel
* ``plan_tables``  the written integer plan rules, implemented independently
                   (``plan_tables_tt`` for kernels in tensor-train form)
* ``tt_full``, ``tt_paths``, ``rhs_dense``  kernels in tensor-train form (Sec. 2):
                   the dense tensor, its rank-path CP factors, and the literal
                   sums from dense kernel tensors
* ``twiddles_ref`` correctly rounded roots of unity via mpmath

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline leg
may import anything from here.  The oracle imports nothing from the product
package and the product package imports nothing from here.
"""
from .native import rhs_direct, rhs_conv, rhs_factored, build_native  # noqa: F401
from .spectral import rhs_fft, total_rhs  # noqa: F401
from .heun import heun_solve, time_grid  # noqa: F401
from .closed_forms import (m0_constant_kernel_d3, m0_rhs_constant_kernel,  # noqa: F401
                           binary_constant_monodisperse, scalar_heun)
from .plan import plan_tables, plan_tables_tt  # noqa: F401
from .tt import tt_full, tt_paths, rhs_dense  # noqa: F401
from .sum_kernel import rhs_sum_kernel  # noqa: F401
