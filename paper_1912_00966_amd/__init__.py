"""MI355X-native earliest-arrival-time (EAT) queries on public-transport timetables.

The package is a thin Python binding over ``libeat.so`` (HIP for gfx950 plus a C++
host preprocessor) whose C ABI is declared in ``include/eat.h``.  Importing the
package loads nothing; the native library is loaded on first use and its absence
is an error, never a fallback.
"""
__all__ = ["synth", "eat"]
