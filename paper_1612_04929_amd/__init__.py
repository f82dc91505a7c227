"""MI355X-native cost and exact gradient for piecewise-constant quantum
optimal control (arXiv:1612.04929), behind the C ABI of ``libqoc.so``.

Import is light: the shared library is loaded on first use by
:func:`paper_1612_04929_amd.qoc.load`, which raises if it is missing.
"""
from . import qoc  # noqa: F401
from .qoc import Problem, QocError, taylor_select, load  # noqa: F401
