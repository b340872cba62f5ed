"""MI355X-native low-rank K-ary quadratic maximizer.

Importing the package is cheap: the HIP library binding lives in
``paper_2602_20376_amd.lrqo`` and is loaded on first use.
"""
