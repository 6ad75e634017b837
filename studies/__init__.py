"""Study drivers (GPU): the precision-form accuracy study, the time-step and
Mach-number error heat maps and the inviscid split-form robustness runs of the
paper's Sec. 4.2, run through the C-ABI.  Each prints one JSON document."""
