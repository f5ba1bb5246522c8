"""Lifetimes in the Python binding (CPU only).

The library calls back into Python through the allocator hook (two ctypes C thunks) whenever a
context, scene or binning allocates or releases device memory, also from a finalizer that runs
during garbage collection.  Two rules keep those calls safe:

  * the thunks are created once, at module level, and live until the process ends (a thunk
    that dies with the object that made it leaves the library a dangling function pointer);
  * the finalizer of a scene or binning holds its Context, so the context (and its handle) is
    destroyed only after everything that releases memory through it.

An earlier binding kept the thunks on each Context and gave the scene and binning finalizers
only the raw handles; a binning collected after its Context called a freed thunk on a destroyed
context.  That happened inside pytest's failure-report formatting (the collection that freed
the failed test's frames ran there) and ended the process with SIGSEGV.
"""
import ctypes
import gc
import weakref

import paper_2507_19718_amd as gsc
from paper_2507_19718_amd import _abi


class _FakeLib:
    def __init__(self):
        self.calls = []

    def gsc_binning_release(self, ctx_handle, h):
        self.calls.append(("binning", ctx_handle, h))

    def gsc_scene_destroy(self, ctx_handle, h):
        self.calls.append(("scene", ctx_handle, h))


class _FakeCtx:
    def __init__(self):
        self._lib = _FakeLib()
        self.handle = ctypes.c_void_p(0x1234)


def test_allocator_thunks_live_at_module_level():
    proto = _abi.gsc_allocator._fields_
    assert isinstance(gsc._ALLOC_FN, proto[0][1]) and isinstance(gsc._RELEASE_FN, proto[1][1])
    # No per-instance thunks: a context's hook struct points at the module's two objects.
    assert not [n for n in vars(gsc.Context) if n in ("_cb", "_callbacks")]


def test_binning_finalizer_keeps_its_context_until_release():
    ctx = _FakeCtx()
    lib = ctx._lib
    ref = weakref.ref(ctx)
    b = gsc.Binning(ctx, ctypes.c_void_p(0x42), 1, None)
    del ctx
    gc.collect()
    assert ref() is not None            # held by the binning's finalizer
    del b
    gc.collect()
    assert lib.calls and lib.calls[0][0] == "binning"
    assert ref() is None                # released after the binning


def test_binning_and_context_in_one_garbage_cycle_release_in_order():
    """The case that crashed: a binning and its context become garbage together, held only by a
    reference cycle (as a failed test's frame is, through its traceback); whatever order the
    collector takes, the release runs while the context is still alive."""
    ctx = _FakeCtx()
    lib = ctx._lib
    b = gsc.Binning(ctx, ctypes.c_void_p(0x43), 1, None)
    frame = {"ctx": ctx, "b": b}
    frame["self"] = frame
    alive_at_release = []
    orig = lib.gsc_binning_release

    def release(ctx_handle, h, _ref=weakref.ref(ctx)):
        alive_at_release.append(_ref() is not None)
        orig(ctx_handle, h)

    lib.gsc_binning_release = release
    del ctx, b, frame
    gc.collect()
    assert alive_at_release == [True]


def test_the_earlier_wiring_released_after_its_context_was_garbage():
    """The mechanism of the crash, on the CPU: a finalizer that holds only the raw handles (as
    the earlier binding's did) lets the context become garbage in the same collection as the
    binning, so when the binning's release runs, the context is already unreachable and its
    own finalizer (destroying the context and, with it, the thunks it owned) may have run."""
    class OldBinning:
        def __init__(self, ctx, handle):
            self._finalizer = weakref.finalize(self, ctx._lib.gsc_binning_release, ctx.handle, handle)

    ctx = _FakeCtx()
    lib = ctx._lib
    b = OldBinning(ctx, ctypes.c_void_p(0x44))
    frame = {"ctx": ctx, "b": b}
    frame["self"] = frame
    alive_at_release = []
    orig = lib.gsc_binning_release
    ref = weakref.ref(ctx)

    def release(ctx_handle, h):
        alive_at_release.append(ref() is not None)
        orig(ctx_handle, h)

    lib.gsc_binning_release = release
    # The finalizer captured the bound method before the swap; route it through the probe.
    b._finalizer.detach()
    b._finalizer = weakref.finalize(b, release, ctx.handle, ctypes.c_void_p(0x44))
    del ctx, b, frame
    gc.collect()
    assert alive_at_release == [False]
